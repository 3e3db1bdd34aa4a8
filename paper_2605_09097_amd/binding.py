"""Python binding of the OS-MPM C ABI (``include/osmpm.h``).

Argument marshalling only: every entry point of ``libosmpm.so`` is exposed
under its C name, PyTorch provides device memory (tensors' ``data_ptr()``)
and the stream (``torch.cuda.current_stream().cuda_stream``).  All work runs
in the library's HIP kernels; if the library is missing this module raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libosmpm.so")

OSMPM_OK, OSMPM_E_INVALID_ARG, OSMPM_E_NO_MEMORY, OSMPM_E_DEVICE = 0, 1, 2, 3
OSMPM_E_OUT_OF_GRID, OSMPM_E_INVERTED, OSMPM_E_NOT_CONVERGED, OSMPM_E_STATE = 4, 5, 6, 7
OSMPM_FP64, OSMPM_MIXED = 0, 1
OSMPM_K_CG_ITER, OSMPM_K_P2G, OSMPM_K_G2P, OSMPM_K_GRAD_HESS = 0, 1, 2, 3

# Every symbol the header declares (checked by the CPU test suite).
ABI_SYMBOLS = [
    "osmpm_ctx_create", "osmpm_ctx_set_stream", "osmpm_ctx_set_graphs", "osmpm_ctx_set_cg_split", "osmpm_sync", "osmpm_last_error", "osmpm_ctx_destroy",
    "osmpm_profile_enable", "osmpm_profile_query",
    "osmpm_domain_create", "osmpm_domain_destroy", "osmpm_domain_set_materials", "osmpm_domain_set_yield",
    "osmpm_domain_set_particles", "osmpm_domain_set_selection", "osmpm_domain_set_scene_bc",
    "osmpm_p2g", "osmpm_implicit_solve", "osmpm_g2p", "osmpm_interface_build",
    "osmpm_project_S_to_B", "osmpm_interp_B_to_S", "osmpm_temporal_interp", "osmpm_set_schwarz_bc",
    "osmpm_schwarz_frame", "osmpm_single_frame", "osmpm_get_particles", "osmpm_get_grid",
    "osmpm_get_sets", "osmpm_get_sort", "osmpm_domain_info",
    "osmpm_batch_create", "osmpm_batch_schwarz_frame", "osmpm_batch_single_frame", "osmpm_batch_destroy",
    "osmpm_multi_create", "osmpm_multi_schwarz_frame",
    "osmpm_single_frame_adjoint", "osmpm_schwarz_frame_adjoint", "osmpm_schwarz_frame_adjoint_implicit",
    "osmpm_single_frame_adjoint_noalloc", "osmpm_batch_run", "osmpm_batch_backward",
]


class osmpm_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int32 * 3), ("h0", C.c_double),
                ("origin_q", C.c_int64 * 3), ("dx_q", C.c_int64)]


class osmpm_material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double)]


class osmpm_solve_opts(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("newton_atol", C.c_double), ("cg_rtol", C.c_double),
                ("max_newton", C.c_int32), ("max_cg", C.c_int32), ("max_ls", C.c_int32),
                ("project_psd", C.c_int32), ("gravity", C.c_double * 3), ("forcing", C.c_double)]


class osmpm_solve_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("cg_iters", C.c_int32), ("ls_halvings", C.c_int32),
                ("converged", C.c_int32), ("ls_failed", C.c_int32), ("gnorm0", C.c_double),
                ("gnorm", C.c_double)]


class osmpm_schwarz_opts(C.Structure):
    _fields_ = [("M", C.c_int32), ("k_max", C.c_int32), ("eps_conv", C.c_double), ("eps_tol", C.c_double),
                ("coarse", osmpm_solve_opts), ("fine", osmpm_solve_opts), ("warm_start", C.c_int32)]


class osmpm_schwarz_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("r_B", C.c_double), ("r_S", C.c_double),
                ("n_recv_B", C.c_int32), ("n_recv_S", C.c_int32), ("n_amb", C.c_int32),
                ("newton_B", C.c_int32), ("newton_S", C.c_int32), ("cg_B", C.c_int32),
                ("cg_S", C.c_int32), ("ls_B", C.c_int32), ("ls_S", C.c_int32),
                ("unconv_B", C.c_int32), ("unconv_S", C.c_int32), ("lsfail_B", C.c_int32),
                ("lsfail_S", C.c_int32)]


_vp = C.c_void_p
_lib = None


def _declare(L):
    st = C.c_int
    P = C.POINTER
    sig = {
        "osmpm_ctx_create": [C.c_int32, _vp, P(_vp)],
        "osmpm_ctx_set_stream": [_vp, _vp],
        "osmpm_ctx_set_graphs": [_vp, C.c_int32],
        "osmpm_ctx_set_cg_split": [_vp, C.c_int32],
        "osmpm_sync": [_vp],
        "osmpm_profile_enable": [_vp, C.c_int32],
        "osmpm_profile_query": [_vp, C.c_int32, P(C.c_int64), P(C.c_double), P(C.c_double)],
        "osmpm_domain_create": [_vp, P(osmpm_grid), C.c_int32, C.c_int64, P(C.c_int32), P(_vp)],
        "osmpm_domain_set_materials": [_vp, P(osmpm_material), C.c_int32],
        "osmpm_domain_set_yield": [_vp, C.c_int32, P(C.c_double)],
        "osmpm_domain_set_particles": [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
        "osmpm_domain_set_selection": [_vp, C.c_double, C.c_double],
        "osmpm_domain_set_scene_bc": [_vp, C.c_int32, P(C.c_int32), P(C.c_int32), P(C.c_double)],
        "osmpm_p2g": [_vp],
        "osmpm_implicit_solve": [_vp, C.c_double, C.c_int32, P(osmpm_solve_opts), P(osmpm_solve_stats)],
        "osmpm_g2p": [_vp, C.c_double],
        "osmpm_interface_build": [_vp, _vp, P(C.c_int32)],
        "osmpm_project_S_to_B": [_vp, _vp, C.c_double, _vp, _vp],
        "osmpm_interp_B_to_S": [_vp, _vp, _vp, _vp],
        "osmpm_temporal_interp": [_vp, C.c_int64, C.c_int32, C.c_int32, _vp, _vp, _vp],
        "osmpm_set_schwarz_bc": [_vp, _vp],
        "osmpm_schwarz_frame": [_vp, _vp, C.c_double, P(osmpm_schwarz_opts), P(osmpm_schwarz_stats)],
        "osmpm_single_frame": [_vp, C.c_double, P(osmpm_solve_opts), P(osmpm_solve_stats)],
        "osmpm_get_particles": [_vp, _vp, _vp, _vp, _vp, _vp],
        "osmpm_get_grid": [_vp, _vp, _vp, _vp],
        "osmpm_get_sets": [_vp, _vp, _vp, _vp],
        "osmpm_get_sort": [_vp, _vp, _vp],
        "osmpm_domain_info": [_vp, P(C.c_int64), P(C.c_int64), P(C.c_int64)],
        "osmpm_batch_create": [_vp, C.c_int32, P(_vp), P(_vp), P(_vp)],
        "osmpm_batch_schwarz_frame": [_vp, C.c_double, P(osmpm_schwarz_opts), P(osmpm_schwarz_stats)],
        "osmpm_batch_single_frame": [_vp, C.c_double, P(osmpm_solve_opts), P(osmpm_solve_stats)],
        "osmpm_multi_create": [_vp, _vp, C.c_int32, P(_vp), P(_vp)],
        "osmpm_multi_schwarz_frame": [_vp, C.c_double, P(osmpm_schwarz_opts), P(osmpm_schwarz_stats)],
        "osmpm_single_frame_adjoint": [_vp, C.c_double, P(osmpm_solve_opts), C.c_double] + [_vp] * 8
                                      + [P(C.c_double)] * 2,
        "osmpm_batch_run": [_vp, C.c_int32, C.c_double, P(osmpm_schwarz_opts), C.c_int32, P(C.c_double),
                            P(osmpm_schwarz_stats)],
        "osmpm_batch_backward": [_vp, P(_vp), P(_vp), C.c_double, C.c_int32, C.c_double, C.c_int32, P(C.c_double)],
        "osmpm_single_frame_adjoint_noalloc": [_vp, C.c_double, P(osmpm_solve_opts), C.c_double] + [_vp] * 8
                                              + [P(C.c_double)] * 2,
        "osmpm_schwarz_frame_adjoint": [_vp, _vp, C.c_double, P(osmpm_schwarz_opts), C.c_int32, C.c_double]
                                       + [_vp] * 16 + [P(C.c_double)] * 4,
        "osmpm_schwarz_frame_adjoint_implicit": [_vp, _vp, C.c_double, P(osmpm_schwarz_opts), C.c_int32,
                                                 C.c_double, C.c_double, C.c_int32, P(C.c_int32)]
                                                + [_vp] * 16 + [P(C.c_double)] * 4,
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.osmpm_last_error.argtypes = [_vp]
    L.osmpm_last_error.restype = C.c_char_p
    L.osmpm_ctx_destroy.argtypes = [_vp]
    L.osmpm_ctx_destroy.restype = None
    L.osmpm_domain_destroy.argtypes = [_vp]
    L.osmpm_domain_destroy.restype = None
    L.osmpm_batch_destroy.argtypes = [_vp]
    L.osmpm_batch_destroy.restype = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libosmpm.so is not built (run __graft_entry__.build() or "
                               "python paper_2605_09097_amd/build.py)")
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


class OsmpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("osmpm status %d: %s" % (status, msg))
        self.status = status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def solve_opts(newton_rtol=1e-8, newton_atol=1e-13, cg_rtol=1e-10, max_newton=50, max_cg=2000, max_ls=30,
               project_psd=True, gravity=(0.0, 0.0, 0.0), forcing=0.0):
    """forcing > 0: Eisenstat-Walker CG tolerances per Newton step, at most
    forcing (see osmpm_solve_opts); 0: cg_rtol alone."""
    o = osmpm_solve_opts()
    o.newton_rtol, o.newton_atol, o.cg_rtol = newton_rtol, newton_atol, cg_rtol
    o.max_newton, o.max_cg, o.max_ls, o.project_psd = max_newton, max_cg, max_ls, int(project_psd)
    o.forcing = forcing
    g = list(gravity) + [0.0] * (3 - len(gravity))
    for a in range(3):
        o.gravity[a] = g[a]
    return o


def schwarz_opts(M, k_max=100, eps_conv=1e-5, eps_tol=0.0, coarse=None, fine=None, warm_start=False):
    o = osmpm_schwarz_opts()
    o.M, o.k_max, o.eps_conv, o.eps_tol = M, k_max, eps_conv, eps_tol
    o.warm_start = int(warm_start)
    o.coarse = coarse if coarse is not None else solve_opts()
    o.fine = fine if fine is not None else solve_opts()
    return o


class Context:
    """osmpm_ctx on a torch device and stream."""

    def __init__(self, device=0, stream=None):
        import torch

        self.torch = torch
        self.device = torch.device("cuda", device)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        h = C.c_void_p()
        st = lib().osmpm_ctx_create(device, C.c_void_p(s.cuda_stream), C.byref(h))
        if st != OSMPM_OK:
            raise OsmpmError(st, "ctx_create")
        self.handle = h

    def check(self, status, what=""):
        if status != OSMPM_OK:
            msg = lib().osmpm_last_error(self.handle)
            raise OsmpmError(status, "%s: %s" % (what, msg.decode() if msg else ""))

    def sync(self):
        self.check(lib().osmpm_sync(self.handle), "sync")

    def graphs(self, enable):
        self.check(lib().osmpm_ctx_set_graphs(self.handle, int(enable)), "set_graphs")

    def cg_split(self, mode):
        """CG scalars inside each CG launch (0), by a launch of their own (1),
        or chosen by size (-1, the default)."""
        self.check(lib().osmpm_ctx_set_cg_split(self.handle, int(mode)), "set_cg_split")

    def profile(self, enable):
        self.check(lib().osmpm_profile_enable(self.handle, int(enable)), "profile_enable")

    def profile_query(self, which):
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        self.check(lib().osmpm_profile_query(self.handle, which, C.byref(n), C.byref(ms), C.byref(by)),
                   "profile_query")
        return n.value, ms.value, by.value

    def temporal_interp(self, m, M, vn, vn1, out):
        self.check(lib().osmpm_temporal_interp(self.handle, vn.numel(), m, M, _ptr(vn), _ptr(vn1), _ptr(out)),
                   "temporal_interp")

    def close(self):
        if self.handle:
            lib().osmpm_ctx_destroy(self.handle)
            self.handle = None


class Domain:
    """osmpm_domain built from a scene domain description (scenes.DomainSpec)."""

    def __init__(self, ctx: Context, spec, precision=OSMPM_FP64, tile=None, capacity=None):
        torch = ctx.torch
        self.ctx = ctx
        self.dim = d = int(spec.dim)
        g = osmpm_grid()
        g.dim = d
        for a in range(3):
            g.n_nodes[a] = int(spec.n_nodes[a]) if a < d else 1
            g.origin_q[a] = int(spec.origin_q[a]) if a < d else 0
        g.h0 = float(spec.h0)
        g.dx_q = int(spec.dx_q)
        self.grid = g
        self.nn = g.n_nodes[0] * g.n_nodes[1] * g.n_nodes[2]
        n = spec.n_particles
        cap = int(capacity if capacity is not None else n)
        t = (C.c_int32 * 3)(*(list(tile) + [0] * (3 - len(tile)))) if tile else None
        h = C.c_void_p()
        ctx.check(lib().osmpm_domain_create(ctx.handle, C.byref(g), precision, cap, t, C.byref(h)),
                  "domain_create")
        self.handle = h
        self.n_mat = len(spec.E)
        mats = (osmpm_material * len(spec.E))(*[osmpm_material(float(E), float(nu))
                                                  for E, nu in zip(spec.E, spec.nu)])
        ctx.check(lib().osmpm_domain_set_materials(h, mats, len(spec.E)), "set_materials")
        ctx.check(lib().osmpm_domain_set_selection(h, float(spec.m_ref), float(spec.tau)), "set_selection")
        if getattr(spec, "tau_y", None) is not None:
            self.set_yield(spec.tau_y)
        self.n_groups = len(spec.bc_kind)
        self._kind = (C.c_int32 * max(self.n_groups, 1))(*spec.bc_kind)
        self._mask = (C.c_int32 * max(self.n_groups, 1))(*spec.bc_mask)
        self.set_bc_params(np.zeros((max(self.n_groups, 1), 8)))
        self.set_particles(spec)

    def set_particles(self, spec):
        torch = self.ctx.torch
        dev = self.ctx.device
        d = self.dim
        n = spec.n_particles
        self._in = [torch.as_tensor(np.ascontiguousarray(a, dtype=dt)).to(dev)
                    for a, dt in ((spec.x, np.float64), (spec.v, np.float64), (spec.B, np.float64),
                                  (spec.F, np.float64), (spec.mass, np.float64), (spec.vol, np.float64),
                                  (spec.mat, np.int32), (spec.flags, np.uint8))]
        x, v, B, F, m, V, mat, fl = self._in
        self.n = n
        self.ctx.check(lib().osmpm_domain_set_particles(self.handle, n, _ptr(x), _ptr(v), _ptr(B), _ptr(F),
                                                        _ptr(m), _ptr(V), _ptr(mat), _ptr(fl)), "set_particles")

    def set_materials(self, E, nu):
        """Young's moduli and Poisson ratios per material (Lame parameters by
        the textbook relations)."""
        mats = (osmpm_material * len(E))(*[osmpm_material(float(a), float(b)) for a, b in zip(E, nu)])
        self.ctx.check(lib().osmpm_domain_set_materials(self.handle, mats, len(E)), "set_materials")
        self.n_mat = len(E)

    def set_yield(self, tau_y):
        """von Mises yield stress per material (<= 0 or inf: elastic); None
        makes every material elastic."""
        if tau_y is None:
            self.ctx.check(lib().osmpm_domain_set_yield(self.handle, 0, None), "set_yield")
            return
        t = np.broadcast_to(np.asarray(tau_y, dtype=np.float64), (self.n_mat,))
        arr = (C.c_double * self.n_mat)(*[float(v) for v in t])
        self.ctx.check(lib().osmpm_domain_set_yield(self.handle, self.n_mat, arr), "set_yield")

    def set_state(self, x, v, B, F):
        """Overwrite the particle state (device tensors in input order) keeping
        masses, volumes, materials and flags of the last set_particles."""
        torch = self.ctx.torch
        xs = [t.to(device=self.ctx.device, dtype=torch.float64).contiguous() for t in (x, v, B, F)]
        _, _, _, _, m, V, mat, fl = self._in
        self._state = xs
        self.ctx.check(lib().osmpm_domain_set_particles(self.handle, self.n, *[_ptr(t) for t in xs], _ptr(m),
                                                        _ptr(V), _ptr(mat), _ptr(fl)), "set_particles")

    def set_bc_params(self, params):
        p = np.zeros((max(self.n_groups, 1), 8))
        params = np.asarray(params, dtype=np.float64)
        if params.size:
            p[: params.shape[0], : params.shape[1]] = params
        arr = (C.c_double * p.size)(*p.ravel())
        self.ctx.check(lib().osmpm_domain_set_scene_bc(self.handle, self.n_groups, self._kind, self._mask, arr),
                       "set_scene_bc")

    # ---- ABI calls ----
    def p2g(self):
        self.ctx.check(lib().osmpm_p2g(self.handle), "p2g")

    def implicit_solve(self, dt, opts, use_schwarz_bc=False):
        st = osmpm_solve_stats()
        self.ctx.check(lib().osmpm_implicit_solve(self.handle, dt, int(use_schwarz_bc), C.byref(opts),
                                                  C.byref(st)), "implicit_solve")
        return st

    def g2p(self, dt):
        self.ctx.check(lib().osmpm_g2p(self.handle, dt), "g2p")

    def single_frame(self, dt, opts):
        st = osmpm_solve_stats()
        self.ctx.check(lib().osmpm_single_frame(self.handle, dt, C.byref(opts), C.byref(st)), "single_frame")
        return st

    def set_schwarz_bc(self, vbc):
        self.ctx.check(lib().osmpm_set_schwarz_bc(self.handle, _ptr(vbc)), "set_schwarz_bc")

    def info(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self.ctx.check(lib().osmpm_domain_info(self.handle, C.byref(a), C.byref(b), C.byref(c)), "info")
        return a.value, b.value, c.value

    # ---- readback (device tensors; .cpu() to inspect) ----
    def particles(self):
        torch = self.ctx.torch
        dev, d, n = self.ctx.device, self.dim, self.n
        x = torch.empty((n, d), dtype=torch.float64, device=dev)
        v = torch.empty((n, d), dtype=torch.float64, device=dev)
        B = torch.empty((n, d, d), dtype=torch.float64, device=dev)
        F = torch.empty((n, d, d), dtype=torch.float64, device=dev)
        i = torch.empty(n, dtype=torch.int32, device=dev)
        self.ctx.check(lib().osmpm_get_particles(self.handle, _ptr(x), _ptr(v), _ptr(B), _ptr(F), _ptr(i)),
                       "get_particles")
        return x, v, B, F, i

    def particles_input_order(self):
        """Particle state as numpy arrays in the order of the input spec."""
        x, v, B, F, i = self.particles()
        self.ctx.sync()
        order = np.argsort(i.cpu().numpy())
        return tuple(t.cpu().numpy()[order] for t in (x, v, B, F))

    def grid_state(self):
        torch = self.ctx.torch
        dev, d = self.ctx.device, self.dim
        m = torch.empty(self.nn, dtype=torch.float64, device=dev)
        vn = torch.empty((self.nn, d), dtype=torch.float64, device=dev)
        u = torch.empty((self.nn, d), dtype=torch.float64, device=dev)
        self.ctx.check(lib().osmpm_get_grid(self.handle, _ptr(m), _ptr(vn), _ptr(u)), "get_grid")
        return m, vn, u

    def sets(self):
        torch = self.ctx.torch
        dev = self.ctx.device
        g = torch.empty(self.nn, dtype=torch.uint8, device=dev)
        r = torch.empty(self.nn, dtype=torch.uint8, device=dev)
        q = torch.empty(self.nn, dtype=torch.int64, device=dev)
        self.ctx.check(lib().osmpm_get_sets(self.handle, _ptr(g), _ptr(r), _ptr(q)), "get_sets")
        return g, r, q

    def sort_result(self):
        torch = self.ctx.torch
        dev = self.ctx.device
        n, _, nk = self.info()
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        cs = torch.empty(nk + 1, dtype=torch.int32, device=dev)
        self.ctx.check(lib().osmpm_get_sort(self.handle, _ptr(perm), _ptr(cs)), "get_sort")
        return perm[:n], cs

    def close(self):
        if self.handle:
            lib().osmpm_domain_destroy(self.handle)
            self.handle = None


def interface_build(B: Domain, S: Domain):
    n = C.c_int32()
    B.ctx.check(lib().osmpm_interface_build(B.handle, S.handle, C.byref(n)), "interface_build")
    return n.value


def project_S_to_B(S: Domain, B: Domain, eps_tol, vS=None, out=None):
    torch = B.ctx.torch
    if out is None:
        out = torch.empty((B.nn, B.dim), dtype=torch.float64, device=B.ctx.device)
    B.ctx.check(lib().osmpm_project_S_to_B(S.handle, B.handle, eps_tol, _ptr(vS), _ptr(out)), "project_S_to_B")
    return out


def interp_B_to_S(B: Domain, S: Domain, vB=None, out=None):
    torch = B.ctx.torch
    if out is None:
        out = torch.empty((S.nn, S.dim), dtype=torch.float64, device=S.ctx.device)
    B.ctx.check(lib().osmpm_interp_B_to_S(B.handle, _ptr(vB), S.handle, _ptr(out)), "interp_B_to_S")
    return out


def schwarz_frame(B: Domain, S: Domain, dT, opts):
    st = osmpm_schwarz_stats()
    B.ctx.check(lib().osmpm_schwarz_frame(B.handle, S.handle, dT, C.byref(opts), C.byref(st)), "schwarz_frame")
    return st


class SchwarzPair:
    """A coarse/fine pair of a scene (scenes.Scene) on one context."""

    def __init__(self, ctx: Context, scene, precision=OSMPM_FP64, tile_B=None, tile_S=None):
        self.scene = scene
        self.B = Domain(ctx, scene.B, precision, tile_B)
        self.S = Domain(ctx, scene.S, precision, tile_S)
        self.frame_index = 0

    def frame(self, opts):
        pB, pS = self.scene.bc_params(self.frame_index)
        self.B.set_bc_params(pB)
        self.S.set_bc_params(pS)
        st = schwarz_frame(self.B, self.S, self.scene.dT, opts)
        self.frame_index += 1
        return st

    def close(self):
        self.B.close()
        self.S.close()


class MultiGroup:
    """One coarse domain and several disjoint fine domains of a scenes.MultiScene
    (osmpm_multi_create / osmpm_multi_schwarz_frame)."""

    def __init__(self, ctx: Context, scene, precision=OSMPM_FP64):
        self.ctx = ctx
        self.scene = scene
        self.B = Domain(ctx, scene.B, precision)
        self.S = [Domain(ctx, s, precision) for s in scene.S]
        k = len(self.S)
        fb = (C.c_void_p * k)(*[d.handle.value for d in self.S])
        h = C.c_void_p()
        ctx.check(lib().osmpm_multi_create(ctx.handle, self.B.handle, k, fb, C.byref(h)), "multi_create")
        self.handle = h
        self.frame_index = 0

    def frame(self, opts):
        pB, pS = self.scene.bc_params(self.frame_index)
        self.B.set_bc_params(pB)
        for D, p in zip(self.S, pS):
            D.set_bc_params(p)
        st = osmpm_schwarz_stats()
        self.ctx.check(lib().osmpm_multi_schwarz_frame(self.handle, self.scene.dT, C.byref(opts), C.byref(st)),
                       "multi_schwarz_frame")
        self.frame_index += 1
        return st

    def close(self):
        if self.handle:
            lib().osmpm_batch_destroy(self.handle)
            self.handle = None
        self.B.close()
        for D in self.S:
            D.close()


class Batch:
    """osmpm_batch over coarse/fine pairs (or single domains when fine is None)."""

    def __init__(self, ctx: Context, coarse, fine=None):
        self.ctx = ctx
        self.n = n = len(coarse)
        if fine is not None and len(fine) != n:
            raise ValueError("coarse and fine lists differ in length")
        cb = (C.c_void_p * n)(*[d.handle.value for d in coarse])
        fb = (C.c_void_p * n)(*[d.handle.value for d in fine]) if fine is not None else None
        h = C.c_void_p()
        ctx.check(lib().osmpm_batch_create(ctx.handle, n, cb, fb, C.byref(h)), "batch_create")
        self.handle = h
        self.coarse, self.fine = list(coarse), (list(fine) if fine is not None else None)

    def schwarz_frame(self, dT, opts):
        st = (osmpm_schwarz_stats * self.n)()
        self.ctx.check(lib().osmpm_batch_schwarz_frame(self.handle, dT, C.byref(opts), st), "batch_schwarz_frame")
        return list(st)

    def single_frame(self, dt, opts):
        st = (osmpm_solve_stats * self.n)()
        self.ctx.check(lib().osmpm_batch_single_frame(self.handle, dt, C.byref(opts), st), "batch_single_frame")
        return list(st)

    def run(self, n_frames, dT, opts, checkpoint_every, bc=None):
        """osmpm_batch_run: n_frames frames; bc is None or a float64 array
        [n_frames][n][2][4][8] of scene-BC parameters.  Returns the frame
        statistics as a list (frames) of lists (pairs)."""
        st = (osmpm_schwarz_stats * (n_frames * self.n))()
        bcp = None
        if bc is not None:
            bc = np.ascontiguousarray(bc, dtype=np.float64)
            if bc.shape != (n_frames, self.n, 2, 4, 8):
                raise ValueError("bc must have shape (n_frames, n, 2, 4, 8)")
            self._bc = bc
            bcp = bc.ctypes.data_as(C.POINTER(C.c_double))
        self.ctx.check(lib().osmpm_batch_run(self.handle, int(n_frames), float(dT), C.byref(opts),
                                             int(checkpoint_every), bcp, st), "batch_run")
        return [list(st[f * self.n:(f + 1) * self.n]) for f in range(n_frames)]

    def backward(self, xbar_B=None, xbar_S=None, adj_cg_rtol=1e-12, implicit=False, fp_tol=1e-10, fp_max=400):
        """osmpm_batch_backward: xbar_B / xbar_S are lists (one entry per pair,
        None for zero) of device float64 tensors [np][d] in input order.
        Returns per pair (dL/dE of the coarse materials, of the fine
        materials) as numpy arrays."""
        keep = []

        def ptrs(lst):
            if lst is None:
                return None
            arr = (C.c_void_p * self.n)()
            for i, t in enumerate(lst):
                if t is not None:
                    t = t.to(dtype=self.ctx.torch.float64).contiguous()
                    keep.append(t)
                    arr[i] = t.data_ptr()
            return arr

        counts = [(b.n_mat, f.n_mat) for b, f in zip(self.coarse, self.fine)]
        out = (C.c_double * sum(a + b for a, b in counts))()
        self.ctx.check(lib().osmpm_batch_backward(self.handle, ptrs(xbar_B), ptrs(xbar_S), float(adj_cg_rtol),
                                                  1 if implicit else 0, float(fp_tol), int(fp_max), out),
                       "batch_backward")
        res, off = [], 0
        for a, b in counts:
            res.append((np.array(out[off:off + a]), np.array(out[off + a:off + a + b])))
            off += a + b
        return res

    def close(self):
        if self.handle:
            lib().osmpm_batch_destroy(self.handle)
            self.handle = None


class SchwarzBatch:
    """Many scenes (scenes.Scene with equal dT and M) as one Schwarz batch."""

    def __init__(self, ctx: Context, scenes_, precision=OSMPM_FP64, tile=None):
        self.scenes = list(scenes_)
        if len({(s.dT, s.M) for s in self.scenes}) != 1:
            raise ValueError("scenes of a batch share dT and M")
        self.dT, self.M = self.scenes[0].dT, self.scenes[0].M
        self.pairs = [SchwarzPair(ctx, s, precision, tile_B=tile, tile_S=tile) for s in self.scenes]
        self.batch = Batch(ctx, [p.B for p in self.pairs], [p.S for p in self.pairs])
        self.frame_index = 0

    def frame(self, opts):
        for p in self.pairs:
            pB, pS = p.scene.bc_params(self.frame_index)
            p.B.set_bc_params(pB)
            p.S.set_bc_params(pS)
            p.frame_index = self.frame_index + 1
        st = self.batch.schwarz_frame(self.dT, opts)
        self.frame_index += 1
        return st

    def bc_table(self, n_frames, first=0):
        """Scene-BC parameters of frames first .. first + n_frames - 1 of every
        scene, in the layout of osmpm_batch_run."""
        bc = np.zeros((n_frames, len(self.pairs), 2, 4, 8))
        for f in range(n_frames):
            for i, p in enumerate(self.pairs):
                for side, prm in enumerate(p.scene.bc_params(first + f)):
                    prm = np.atleast_2d(np.asarray(prm, dtype=np.float64))
                    bc[f, i, side, :prm.shape[0], :prm.shape[1]] = prm
        return bc

    def run(self, n_frames, opts, checkpoint_every=10):
        """n_frames frames from the current frame index in one osmpm_batch_run
        (kept for backward)."""
        st = self.batch.run(n_frames, self.dT, opts, checkpoint_every, self.bc_table(n_frames, self.frame_index))
        self.frame_index += n_frames
        for p in self.pairs:
            p.frame_index = self.frame_index
        return st

    def backward(self, xbar_B=None, xbar_S=None, **kw):
        return self.batch.backward(xbar_B, xbar_S, **kw)

    def close(self):
        self.batch.close()
        for p in self.pairs:
            p.close()


# ---------------------------------------------------------------- reverse mode
def _adj_in(D, adj):
    """Device FP64 copies of an adjoint state dict (zeros where absent), in
    the caller's layout and input particle order."""
    torch = D.ctx.torch
    dev, d, n = D.ctx.device, D.dim, D.n
    out = []
    for k, shape in (("x", (n, d)), ("v", (n, d)), ("B", (n, d, d)), ("F", (n, d, d))):
        a = None if adj is None else adj.get(k)
        t = torch.zeros(shape, dtype=torch.float64, device=dev) if a is None else \
            torch.as_tensor(np.asarray(a, dtype=np.float64) if not hasattr(a, "device") else a).to(
                device=dev, dtype=torch.float64).reshape(shape).contiguous()
        out.append(t)
    return out


def _adj_out(D):
    torch = D.ctx.torch
    dev, d, n = D.ctx.device, D.dim, D.n
    return [torch.zeros(s, dtype=torch.float64, device=dev) for s in ((n, d), (n, d), (n, d, d), (n, d, d))]


def single_frame_adjoint(D: Domain, dt, opts, adj_end, adj_cg_rtol=1e-12, noalloc=False):
    """Adjoint of one single-domain frame from D's current state (see
    osmpm_single_frame_adjoint; noalloc=True calls
    osmpm_single_frame_adjoint_noalloc).  Returns ({x, v, B, F} adjoint of the
    start state as device tensors, dL/dmu, dL/dlam per material as numpy
    arrays)."""
    a = _adj_in(D, adj_end)
    o = _adj_out(D)
    nm = D.n_mat
    mub = (C.c_double * nm)()
    lab = (C.c_double * nm)()
    fn = lib().osmpm_single_frame_adjoint_noalloc if noalloc else lib().osmpm_single_frame_adjoint
    D.ctx.check(fn(D.handle, dt, C.byref(opts), adj_cg_rtol, *[_ptr(t) for t in a], *[_ptr(t) for t in o], mub,
                   lab), "single_frame_adjoint" + ("_noalloc" if noalloc else ""))
    return dict(zip("xvBF", o)), np.array(mub[:]), np.array(lab[:])


def schwarz_frame_adjoint(B: Domain, S: Domain, dT, opts, iters, adjB_end, adjS_end, adj_cg_rtol=1e-12):
    """Adjoint of one Schwarz frame with `iters` iterations from the pair's
    current states (see osmpm_schwarz_frame_adjoint).  Returns (adjoint of
    B's start state, of S's start state, dL/dmu_B, dL/dlam_B, dL/dmu_S,
    dL/dlam_S)."""
    aB, aS = _adj_in(B, adjB_end), _adj_in(S, adjS_end)
    oB, oS = _adj_out(B), _adj_out(S)
    mB, lB = (C.c_double * B.n_mat)(), (C.c_double * B.n_mat)()
    mS, lS = (C.c_double * S.n_mat)(), (C.c_double * S.n_mat)()
    B.ctx.check(lib().osmpm_schwarz_frame_adjoint(B.handle, S.handle, dT, C.byref(opts), int(iters), adj_cg_rtol,
                                                  *[_ptr(t) for t in aB], *[_ptr(t) for t in aS],
                                                  *[_ptr(t) for t in oB], *[_ptr(t) for t in oS], mB, lB, mS, lS),
                "schwarz_frame_adjoint")
    return (dict(zip("xvBF", oB)), dict(zip("xvBF", oS)), np.array(mB[:]), np.array(lB[:]), np.array(mS[:]),
            np.array(lS[:]))


def schwarz_frame_adjoint_implicit(B: Domain, S: Domain, dT, opts, iters, adjB_end, adjS_end, fp_tol=1e-10,
                                   fp_max=200, adj_cg_rtol=1e-12):
    """Implicit (fixed-point) adjoint of one Schwarz frame from the pair's
    current states (see osmpm_schwarz_frame_adjoint_implicit).  Returns the
    tuple of schwarz_frame_adjoint plus the number of adjoint passes."""
    aB, aS = _adj_in(B, adjB_end), _adj_in(S, adjS_end)
    oB, oS = _adj_out(B), _adj_out(S)
    mB, lB = (C.c_double * B.n_mat)(), (C.c_double * B.n_mat)()
    mS, lS = (C.c_double * S.n_mat)(), (C.c_double * S.n_mat)()
    used = C.c_int32(0)
    B.ctx.check(lib().osmpm_schwarz_frame_adjoint_implicit(
        B.handle, S.handle, dT, C.byref(opts), int(iters), adj_cg_rtol, float(fp_tol), int(fp_max), C.byref(used),
        *[_ptr(t) for t in aB], *[_ptr(t) for t in aS], *[_ptr(t) for t in oB], *[_ptr(t) for t in oS],
        mB, lB, mS, lS), "schwarz_frame_adjoint_implicit")
    return (dict(zip("xvBF", oB)), dict(zip("xvBF", oS)), np.array(mB[:]), np.array(lB[:]), np.array(mS[:]),
            np.array(lS[:]), used.value)
