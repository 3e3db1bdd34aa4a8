"""FP64 CPU oracle of OS-MPM (arXiv 2605.09097) -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``oracle.c``: the plain, slow, single-threaded
double-precision implementation of the method that the GPU library is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It imports
nothing from the GPU package and the GPU package imports nothing from it.

Every routine here follows a section or equation of the paper; the C source
names them.  The Lame parameters are computed here from (E, nu) with the
textbook relations mu = E / (2 (1 + nu)), lam = E nu / ((1 + nu)(1 - 2 nu)).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_FIX, BC_TRANSLATE, BC_ROTATE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no threads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_u8p = C.POINTER(C.c_ubyte)
_i8p = C.POINTER(C.c_byte)
_i64p = C.POINTER(C.c_longlong)


class _Domain(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n", C.c_int * 3), ("h0", C.c_double),
        ("origin_q", C.c_longlong * 3), ("dx_q", C.c_longlong),
        ("np", C.c_int), ("x", _dp), ("v", _dp), ("B", _dp), ("F", _dp),
        ("mass", _dp), ("vol", _dp), ("mat", _ip), ("flags", _u8p),
        ("n_mat", C.c_int), ("mu", _dp), ("lam", _dp),
        ("n_groups", C.c_int), ("bc_kind", _ip), ("bc_mask", _ip), ("bc_param", _dp),
        ("m_ref", C.c_double), ("tau", C.c_double),
        ("m", _dp), ("vn", _dp), ("u", _dp), ("bcg", _i8p), ("q_all", _i64p),
        ("q_bnd", _i64p), ("gamma", _u8p), ("recv", _u8p), ("vbc", _dp),
        ("use_schwarz_bc", C.c_int), ("tau_y", _dp),
    ]


class SolveOpts(C.Structure):
    _fields_ = [
        ("newton_rtol", C.c_double), ("newton_atol", C.c_double), ("cg_rtol", C.c_double),
        ("max_newton", C.c_int), ("max_cg", C.c_int), ("max_ls", C.c_int),
        ("project_psd", C.c_int), ("gravity", C.c_double * 3),
    ]


class SolveStats(C.Structure):
    _fields_ = [
        ("newton_iters", C.c_int), ("cg_iters", C.c_int), ("ls_halvings", C.c_int),
        ("converged", C.c_int), ("ls_failed", C.c_int),
        ("gnorm0", C.c_double), ("gnorm", C.c_double), ("energy", C.c_double),
    ]


class SchwarzOpts(C.Structure):
    _fields_ = [
        ("M", C.c_int), ("k_max", C.c_int), ("eps_conv", C.c_double), ("eps_tol", C.c_double),
        ("coarse", SolveOpts), ("fine", SolveOpts), ("force_iters", C.c_int), ("warm_start", C.c_int),
    ]


class SchwarzStats(C.Structure):
    _fields_ = [
        ("iters", C.c_int), ("converged", C.c_int), ("r_B", C.c_double), ("r_S", C.c_double),
        ("n_recv_B", C.c_int), ("n_recv_S", C.c_int), ("n_amb", C.c_int),
        ("newton_B", C.c_int), ("newton_S", C.c_int), ("cg_B", C.c_int), ("cg_S", C.c_int),
        ("ls_B", C.c_int), ("ls_S", C.c_int),
        ("unconv_B", C.c_int), ("unconv_S", C.c_int), ("lsfail_B", C.c_int), ("lsfail_S", C.c_int),
    ]


def _declare(L):
    dom = C.POINTER(_Domain)
    L.or_weights.argtypes = [dom, _dp, _ip, _dp, _dp]
    L.or_num_keys.argtypes = [dom, _ip]
    L.or_num_keys.restype = C.c_longlong
    L.or_sort.argtypes = [dom, _ip, _ip, _ip]
    L.or_p2g.argtypes = [dom]
    L.or_nh_eval.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _dp, _dp, _dp, C.c_int]
    L.or_psd_project.argtypes = [_dp, C.c_int]
    L.or_vm_return.argtypes = [C.c_int, _dp, C.c_double, C.c_double]
    L.or_energy.argtypes = [dom, C.c_double, _dp, _dp, _dp]
    L.or_delta_energy.argtypes = [dom, C.c_double, _dp, _dp, _dp, C.c_double, _dp]
    L.or_gradient.argtypes = [dom, C.c_double, _dp, _dp, _dp]
    L.or_hvp.argtypes = [dom, C.c_double, _dp, _dp, C.c_int, _dp, _dp]
    L.or_dirichlet.argtypes = [dom, C.c_double, _u8p, _dp]
    L.or_solve.argtypes = [dom, C.c_double, C.POINTER(SolveOpts), C.POINTER(SolveStats)]
    L.or_g2p.argtypes = [dom, C.c_double]
    L.or_interface.argtypes = [dom, dom, _ip]
    L.or_project.argtypes = [dom, dom, C.c_double, _dp, _dp]
    L.or_interp.argtypes = [dom, _dp, dom, _dp]
    L.or_temporal.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
    L.or_temporal.restype = None
    L.or_single_frame.argtypes = [dom, C.c_double, C.POINTER(SolveOpts), C.POINTER(SolveStats)]
    L.or_schwarz_frame.argtypes = [dom, dom, C.c_double, C.POINTER(SchwarzOpts),
                                   C.POINTER(SchwarzStats)]
    L.or_schwarz_frame_multi.argtypes = [dom, C.POINTER(dom), C.c_int, C.c_double, C.POINTER(SchwarzOpts),
                                         C.POINTER(SchwarzStats)]
    L.or_single_frame_adjoint.argtypes = [dom, C.c_double, C.POINTER(SolveOpts), C.c_double] + [_dp] * 10
    L.or_schwarz_frame_adjoint.argtypes = ([dom, dom, C.c_double, C.POINTER(SchwarzOpts), C.c_int, C.c_double]
                                           + [_dp] * 20)
    L.or_schwarz_frame_adjoint_implicit.argtypes = ([dom, dom, C.c_double, C.POINTER(SchwarzOpts), C.c_int,
                                                     C.c_double, C.c_double, C.c_int, C.POINTER(C.c_int)]
                                                    + [_dp] * 20)


def _ptr(a, t):
    return a.ctypes.data_as(t)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError("%s failed with status %d" % (what, rc))


def lame(E, nu):
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


class Domain:
    """One subdomain held in numpy arrays (particle state is updated in place).

    ``spec`` is any object with the attributes of a scene domain description:
    dim, h0, origin_q, dx_q, n_nodes, x, v, B, F, mass, vol, mat, flags, E, nu,
    bc_kind, bc_mask, m_ref, tau.
    """

    def __init__(self, spec):
        d = int(spec.dim)
        self.dim = d
        n = [int(k) for k in spec.n_nodes] + [1] * (3 - d)
        self.n = n
        self.nn = n[0] * n[1] * n[2]
        self.x = np.ascontiguousarray(spec.x, dtype=np.float64).reshape(-1, d).copy()
        npart = self.x.shape[0]
        self.v = np.ascontiguousarray(spec.v, dtype=np.float64).reshape(npart, d).copy()
        self.B = np.ascontiguousarray(spec.B, dtype=np.float64).reshape(npart, d, d).copy()
        self.F = np.ascontiguousarray(spec.F, dtype=np.float64).reshape(npart, d, d).copy()
        self.mass = np.ascontiguousarray(spec.mass, dtype=np.float64).copy()
        self.vol = np.ascontiguousarray(spec.vol, dtype=np.float64).copy()
        self.mat = np.ascontiguousarray(spec.mat, dtype=np.int32).copy()
        self.flags = np.ascontiguousarray(spec.flags, dtype=np.uint8).copy()
        mu, lam = lame(spec.E, spec.nu)
        self.mu = np.ascontiguousarray(np.atleast_1d(mu), dtype=np.float64)
        self.lam = np.ascontiguousarray(np.atleast_1d(lam), dtype=np.float64)
        ng = len(spec.bc_kind)
        self.bc_kind = np.ascontiguousarray(np.asarray(spec.bc_kind, dtype=np.int32).reshape(ng) if ng else np.zeros(1, np.int32))
        self.bc_mask = np.ascontiguousarray(np.asarray(spec.bc_mask, dtype=np.int32).reshape(ng) if ng else np.zeros(1, np.int32))
        self.bc_param = np.zeros((max(ng, 1), 8), dtype=np.float64)
        self.m = np.zeros(self.nn)
        self.vn = np.zeros((self.nn, d))
        self.u = np.zeros((self.nn, d))
        self.bcg = np.full((self.nn, d), -1, dtype=np.int8)
        self.q_all = np.zeros(self.nn, dtype=np.int64)
        self.q_bnd = np.zeros(self.nn, dtype=np.int64)
        self.gamma = np.zeros(self.nn, dtype=np.uint8)
        self.recv = np.zeros(self.nn, dtype=np.uint8)
        self.vbc = np.zeros((self.nn, d))
        s = _Domain()
        s.dim = d
        for a in range(3):
            s.n[a] = n[a]
            s.origin_q[a] = int(spec.origin_q[a]) if a < d else 0
        s.h0 = float(spec.h0)
        s.dx_q = int(spec.dx_q)
        s.np = npart
        s.x, s.v, s.B, s.F = (_ptr(self.x, _dp), _ptr(self.v, _dp), _ptr(self.B, _dp),
                              _ptr(self.F, _dp))
        s.mass, s.vol = _ptr(self.mass, _dp), _ptr(self.vol, _dp)
        s.mat, s.flags = _ptr(self.mat, _ip), _ptr(self.flags, _u8p)
        s.n_mat = len(self.mu)
        s.mu, s.lam = _ptr(self.mu, _dp), _ptr(self.lam, _dp)
        s.n_groups = ng
        s.bc_kind, s.bc_mask = _ptr(self.bc_kind, _ip), _ptr(self.bc_mask, _ip)
        s.bc_param = _ptr(self.bc_param, _dp)
        s.m_ref, s.tau = float(spec.m_ref), float(spec.tau)
        s.m, s.vn, s.u = _ptr(self.m, _dp), _ptr(self.vn, _dp), _ptr(self.u, _dp)
        s.bcg = _ptr(self.bcg, _i8p)
        s.q_all, s.q_bnd = _ptr(self.q_all, _i64p), _ptr(self.q_bnd, _i64p)
        s.gamma, s.recv = _ptr(self.gamma, _u8p), _ptr(self.recv, _u8p)
        s.vbc = _ptr(self.vbc, _dp)
        s.use_schwarz_bc = 0
        self._s = s
        self.tau_y = None
        ty = getattr(spec, "tau_y", None)
        if ty is not None:
            self.set_yield(ty)

    # -- state helpers -------------------------------------------------
    @property
    def ref(self):
        return C.byref(self._s)

    def set_bc_params(self, params):
        params = np.asarray(params, dtype=np.float64)
        if params.size:
            self.bc_param[: params.shape[0], : params.shape[1]] = params

    def state(self):
        return {"x": self.x.copy(), "v": self.v.copy(), "B": self.B.copy(), "F": self.F.copy()}

    def set_state(self, st):
        """Overwrite the particle state in place (arrays keep their addresses)."""
        for k in ("x", "v", "B", "F"):
            getattr(self, k)[...] = st[k]

    def set_yield(self, tau_y):
        """von Mises yield stress per material (<= 0 or inf: elastic); None
        makes every material elastic."""
        if tau_y is None:
            self.tau_y = None
            self._s.tau_y = _dp()
            return
        self.tau_y = np.ascontiguousarray(np.broadcast_to(np.asarray(tau_y, dtype=np.float64), self.mu.shape)).copy()
        self._s.tau_y = _ptr(self.tau_y, _dp)

    def set_lame(self, mu, lam):
        self.mu[...] = mu
        self.lam[...] = lam

    def node_positions(self):
        d = self.dim
        idx = np.indices(self.n[:d][::-1]).reshape(d, -1)[::-1].T  # x fastest
        o = np.array(self._s.origin_q[:d], dtype=np.int64)
        return ((o + idx.astype(np.int64) * self._s.dx_q).astype(np.float64)) * self._s.h0

    # -- method pieces ---------------------------------------------------
    def weights(self, xp):
        ss = 27 if self.dim == 3 else 9
        flat = np.zeros(ss, dtype=np.int32)
        N = np.zeros(ss)
        gN = np.zeros((ss, 3))
        xp = np.ascontiguousarray(xp, dtype=np.float64)
        _check(lib().or_weights(self.ref, _ptr(xp, _dp), _ptr(flat, _ip), _ptr(N, _dp),
                                _ptr(gN, _dp)), "or_weights")
        return flat, N, gN[:, : self.dim]

    def sort(self, tile):
        t = np.ascontiguousarray(list(tile) + [1] * (3 - len(tile)), dtype=np.int32)
        nk = lib().or_num_keys(self.ref, _ptr(t, _ip))
        perm = np.zeros(self.x.shape[0], dtype=np.int32)
        cs = np.zeros(nk + 1, dtype=np.int32)
        _check(lib().or_sort(self.ref, _ptr(t, _ip), _ptr(perm, _ip), _ptr(cs, _ip)), "or_sort")
        return perm, cs

    def p2g(self):
        _check(lib().or_p2g(self.ref), "or_p2g")

    def energy(self, dt, u, gravity=(0, 0, 0)):
        g = np.ascontiguousarray(list(gravity) + [0] * (3 - len(gravity)), dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros(1)
        _check(lib().or_energy(self.ref, dt, _ptr(g, _dp), _ptr(u, _dp), _ptr(out, _dp)),
               "or_energy")
        return float(out[0])

    def delta_energy(self, dt, u, du, alpha, gravity=(0, 0, 0)):
        g = np.ascontiguousarray(list(gravity) + [0] * (3 - len(gravity)), dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        du = np.ascontiguousarray(du, dtype=np.float64)
        out = np.zeros(1)
        _check(lib().or_delta_energy(self.ref, dt, _ptr(g, _dp), _ptr(u, _dp), _ptr(du, _dp),
                                     alpha, _ptr(out, _dp)), "or_delta_energy")
        return float(out[0])

    def gradient(self, dt, u, gravity=(0, 0, 0)):
        g = np.ascontiguousarray(list(gravity) + [0] * (3 - len(gravity)), dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros_like(u)
        _check(lib().or_gradient(self.ref, dt, _ptr(g, _dp), _ptr(u, _dp), _ptr(out, _dp)),
               "or_gradient")
        return out

    def hvp(self, dt, u, w, project=False):
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        y = np.zeros_like(u)
        dg = np.zeros_like(u)
        _check(lib().or_hvp(self.ref, dt, _ptr(u, _dp), _ptr(w, _dp), int(project),
                            _ptr(y, _dp), _ptr(dg, _dp)), "or_hvp")
        return y, dg

    def dirichlet(self, dt):
        dr = np.zeros((self.nn, self.dim), dtype=np.uint8)
        ud = np.zeros((self.nn, self.dim))
        _check(lib().or_dirichlet(self.ref, dt, _ptr(dr, _u8p), _ptr(ud, _dp)), "or_dirichlet")
        return dr, ud

    def solve(self, dt, opts, use_schwarz_bc=False):
        self._s.use_schwarz_bc = int(use_schwarz_bc)
        st = SolveStats()
        _check(lib().or_solve(self.ref, dt, C.byref(opts), C.byref(st)), "or_solve")
        return st

    def g2p(self, dt):
        _check(lib().or_g2p(self.ref, dt), "or_g2p")

    def single_frame(self, dt, opts):
        st = SolveStats()
        _check(lib().or_single_frame(self.ref, dt, C.byref(opts), C.byref(st)),
               "or_single_frame")
        return st


def nh_eval(F, mu, lam, project=False):
    F = np.ascontiguousarray(F, dtype=np.float64)
    d = F.shape[0]
    psi = np.zeros(1)
    P = np.zeros((d, d))
    A = np.zeros((d * d, d * d))
    rc = lib().or_nh_eval(d, _ptr(F, _dp), mu, lam, _ptr(psi, _dp), _ptr(P, _dp), _ptr(A, _dp),
                          int(project))
    return float(psi[0]), P, A, rc


def vm_return(F, mu, tau_y):
    """The von Mises return in Hencky strain applied to one deformation
    gradient (returns the projected F and whether it changed)."""
    F = np.ascontiguousarray(F, dtype=np.float64).copy()
    rc = lib().or_vm_return(F.shape[0], _ptr(F, _dp), mu, tau_y)
    if rc < 0:
        raise ValueError("dimension")
    return F, bool(rc)


def psd_project(A):
    A = np.ascontiguousarray(A, dtype=np.float64).copy()
    _check(lib().or_psd_project(_ptr(A, _dp), A.shape[0]), "or_psd_project")
    return A


def interface(Bd: Domain, Sd: Domain):
    n_amb = np.zeros(1, dtype=np.int32)
    _check(lib().or_interface(Bd.ref, Sd.ref, _ptr(n_amb, _ip)), "or_interface")
    return int(n_amb[0])


def project(Sd: Domain, Bd: Domain, eps_tol, vS=None):
    vS = np.ascontiguousarray(Sd.vn if vS is None else vS, dtype=np.float64)
    out = np.zeros((Bd.nn, Bd.dim))
    _check(lib().or_project(Sd.ref, Bd.ref, eps_tol, _ptr(vS, _dp), _ptr(out, _dp)),
           "or_project")
    return out


def interp(Bd: Domain, vB, Sd: Domain):
    vB = np.ascontiguousarray(vB, dtype=np.float64)
    out = np.zeros((Sd.nn, Sd.dim))
    _check(lib().or_interp(Bd.ref, _ptr(vB, _dp), Sd.ref, _ptr(out, _dp)), "or_interp")
    return out


def temporal(m, M, vn, vn1):
    vn = np.ascontiguousarray(vn, dtype=np.float64)
    vn1 = np.ascontiguousarray(vn1, dtype=np.float64)
    out = np.zeros_like(vn)
    lib().or_temporal(vn.size, m, M, _ptr(vn, _dp), _ptr(vn1, _dp), _ptr(out, _dp))
    return out


def solve_opts(newton_rtol=1e-8, newton_atol=1e-13, cg_rtol=1e-10, max_newton=50, max_cg=2000,
               max_ls=30, project_psd=True, gravity=(0.0, 0.0, 0.0)):
    o = SolveOpts()
    o.newton_rtol, o.newton_atol, o.cg_rtol = newton_rtol, newton_atol, cg_rtol
    o.max_newton, o.max_cg, o.max_ls = max_newton, max_cg, max_ls
    o.project_psd = int(project_psd)
    g = list(gravity) + [0.0] * (3 - len(gravity))
    for a in range(3):
        o.gravity[a] = g[a]
    return o


def schwarz_opts(M, k_max=100, eps_conv=1e-5, eps_tol=0.0, coarse=None, fine=None, force_iters=0,
                 warm_start=False):
    o = SchwarzOpts()
    o.warm_start = int(warm_start)
    o.M, o.k_max, o.eps_conv, o.eps_tol = M, k_max, eps_conv, eps_tol
    o.force_iters = int(force_iters)
    o.coarse = coarse if coarse is not None else solve_opts()
    o.fine = fine if fine is not None else solve_opts()
    return o


def schwarz_frame(Bd: Domain, Sd: Domain, dT, opts):
    st = SchwarzStats()
    _check(lib().or_schwarz_frame(Bd.ref, Sd.ref, dT, C.byref(opts), C.byref(st)),
           "or_schwarz_frame")
    return st


def schwarz_frame_multi(Bd: Domain, Sds, dT, opts):
    """One frame of Alg. 1 with the coarse domain Bd and the disjoint fine
    domains Sds (or_schwarz_frame_multi)."""
    st = SchwarzStats()
    arr = (C.POINTER(_Domain) * len(Sds))(*[C.pointer(S._s) for S in Sds])
    _check(lib().or_schwarz_frame_multi(Bd.ref, arr, len(Sds), dT, C.byref(opts), C.byref(st)),
           "or_schwarz_frame_multi")
    return st


# ---------------------------------------------------------------- reverse mode
def _adj_arrays(D, adj):
    """Contiguous float64 copies of an adjoint state dict (zeros where absent)."""
    out = {}
    for k, shape in (("x", D.x.shape), ("v", D.v.shape), ("B", D.B.shape), ("F", D.F.shape)):
        a = adj.get(k) if adj is not None else None
        out[k] = np.ascontiguousarray(np.zeros(shape) if a is None else np.asarray(a, dtype=np.float64).reshape(shape))
    return out


def single_frame_adjoint(D: Domain, dt, opts, adj_end, adj_cg_rtol=1e-13):
    """Adjoint of one single-domain frame.  D holds the start-of-frame state
    (on exit: the end state, the frame being recomputed).  adj_end: adjoint
    of the end state ({x, v, B, F}).  Returns (adjoint of the start state,
    dL/dmu, dL/dlam per material)."""
    a = _adj_arrays(D, adj_end)
    o = {k: np.zeros_like(v) for k, v in a.items()}
    mub = np.zeros_like(D.mu)
    lab = np.zeros_like(D.lam)
    _check(lib().or_single_frame_adjoint(D.ref, dt, C.byref(opts), adj_cg_rtol,
                                         *[_ptr(a[k], _dp) for k in "xvBF"], *[_ptr(o[k], _dp) for k in "xvBF"],
                                         _ptr(mub, _dp), _ptr(lab, _dp)), "or_single_frame_adjoint")
    return o, mub, lab


def schwarz_frame_adjoint(Bd: Domain, Sd: Domain, dT, opts, iters, adjB_end, adjS_end, adj_cg_rtol=1e-13):
    """Adjoint of one Schwarz frame with `iters` Schwarz iterations (the
    forward's count).  Bd, Sd hold the start-of-frame states (on exit the end
    states).  Returns (adjoint of B's start state, of S's start state,
    dL/dmu_B, dL/dlam_B, dL/dmu_S, dL/dlam_S), the material adjoints per
    material index of each domain."""
    aB = _adj_arrays(Bd, adjB_end)
    aS = _adj_arrays(Sd, adjS_end)
    oB = {k: np.zeros_like(v) for k, v in aB.items()}
    oS = {k: np.zeros_like(v) for k, v in aS.items()}
    mubB, labB = np.zeros_like(Bd.mu), np.zeros_like(Bd.lam)
    mubS, labS = np.zeros_like(Sd.mu), np.zeros_like(Sd.lam)
    _check(lib().or_schwarz_frame_adjoint(
        Bd.ref, Sd.ref, dT, C.byref(opts), int(iters), adj_cg_rtol,
        *[_ptr(aB[k], _dp) for k in "xvBF"], *[_ptr(aS[k], _dp) for k in "xvBF"],
        *[_ptr(oB[k], _dp) for k in "xvBF"], *[_ptr(oS[k], _dp) for k in "xvBF"],
        _ptr(mubB, _dp), _ptr(labB, _dp), _ptr(mubS, _dp), _ptr(labS, _dp)), "or_schwarz_frame_adjoint")
    return oB, oS, mubB, labB, mubS, labS


def schwarz_frame_adjoint_implicit(Bd: Domain, Sd: Domain, dT, opts, iters, adjB_end, adjS_end, fp_tol=1e-10,
                                   fp_max=200, adj_cg_rtol=1e-13):
    """Implicit (fixed-point) adjoint of one Schwarz frame: the Neumann series
    of the adjoint iteration at the last forward iterate, with no term from
    the first iterate's data (or_schwarz_frame_adjoint_implicit).  Returns the
    tuple of schwarz_frame_adjoint plus the number of adjoint passes."""
    aB = _adj_arrays(Bd, adjB_end)
    aS = _adj_arrays(Sd, adjS_end)
    oB = {k: np.zeros_like(v) for k, v in aB.items()}
    oS = {k: np.zeros_like(v) for k, v in aS.items()}
    mubB, labB = np.zeros_like(Bd.mu), np.zeros_like(Bd.lam)
    mubS, labS = np.zeros_like(Sd.mu), np.zeros_like(Sd.lam)
    used = C.c_int(0)
    _check(lib().or_schwarz_frame_adjoint_implicit(
        Bd.ref, Sd.ref, dT, C.byref(opts), int(iters), adj_cg_rtol, float(fp_tol), int(fp_max), C.byref(used),
        *[_ptr(aB[k], _dp) for k in "xvBF"], *[_ptr(aS[k], _dp) for k in "xvBF"],
        *[_ptr(oB[k], _dp) for k in "xvBF"], *[_ptr(oS[k], _dp) for k in "xvBF"],
        _ptr(mubB, _dp), _ptr(labB, _dp), _ptr(mubS, _dp), _ptr(labS, _dp)), "or_schwarz_frame_adjoint_implicit")
    return oB, oS, mubB, labB, mubS, labS, used.value


def schwarz_run(scene, E, n_frames, opts):
    """Runs frames 0 .. n_frames-1 of a scene pair with Young's moduli E (the
    fine domain's material list; the coarse one's is its prefix).  Returns
    (B, S, per-frame start states, per-frame Schwarz iteration counts)."""
    Bd, Sd = Domain(scene.B), Domain(scene.S)
    nB = len(scene.B.E)
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(scene.S.nu, dtype=np.float64)
    mu, lam = lame(E, nu)
    Bd.set_lame(mu[:nB], lam[:nB])
    Sd.set_lame(mu, lam)
    starts, iters = [], []
    for f in range(n_frames):
        starts.append((Bd.state(), Sd.state()))
        pB, pS = scene.bc_params(f)
        Bd.set_bc_params(pB)
        Sd.set_bc_params(pS)
        iters.append(schwarz_frame(Bd, Sd, scene.dT, opts).iters)
    return Bd, Sd, starts, iters


def schwarz_run_gradient(scene, E, Bd, Sd, starts, iters, opts, adjB_end, adjS_end=None):
    """Reverse sweep over the frames of schwarz_run (frame adjoints from the
    stored start states, last frame first).  Returns (dL/dE per material,
    adjoint of the initial coarse state, of the initial fine state)."""
    nB = len(scene.B.E)
    nu = np.asarray(scene.S.nu, dtype=np.float64)
    dmu = 1.0 / (2.0 * (1.0 + nu))
    dlam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    dE = np.zeros(len(nu))
    aB, aS = adjB_end, adjS_end
    for f in range(len(iters) - 1, -1, -1):
        Bd.set_state(starts[f][0])
        Sd.set_state(starts[f][1])
        pB, pS = scene.bc_params(f)
        Bd.set_bc_params(pB)
        Sd.set_bc_params(pS)
        aB, aS, mB, lB, mS, lS = schwarz_frame_adjoint(Bd, Sd, scene.dT, opts, iters[f], aB, aS)
        dE[:nB] += mB * dmu[:nB] + lB * dlam[:nB]
        dE += mS * dmu + lS * dlam
    return dE, aB, aS
