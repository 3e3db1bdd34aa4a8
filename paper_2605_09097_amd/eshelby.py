"""Efficiency study on the elastic inclusion (Sec. 4.3): OS-MPM against the
single-domain fine discretisation, both run to static equilibrium on the GPU,
with the stress error measured against the plane-strain Eshelby solution.

Setup (readings of Sec. 4.3 where it is silent): unit-square layout of the
inclusion scenes (matrix [0.1, 0.9]^2, inclusion radius R = 0.05, fine
domain r <= 0.15 on [0.3, 0.7]^2, coarse domain outside r = 0.1), matrix
E = 1e5 Pa, nu = 0.3 in both materials, misfit F0 = (1 - delta) I with
delta = 0.01 in the inclusion, 2 x 2 particles per cell.  The outer edge of
the matrix square is clamped: with a traction-free edge the two-domain run
does not conserve momentum (Dirichlet-Dirichlet coupling) and the whole body
drifts, so the equilibrium criterion is never met.  The single-domain run
uses cell size h and dt = 0.01 s at h = 1/50 with dt / h fixed; OS-MPM uses h
on the fine domain, 2h on the coarse one, dT = 2 dt (M = 2).  Both stop when
the l-infinity norm of the grid velocity is below 1e-6 on every grid.

Stress: Cauchy stress sigma = P F^T / J of each particle (plane strain,
Neo-Hookean P), compared with the exact field -P_c I inside r < R and
sigma_rr = -P_c (R/r)^2, sigma_tt = +P_c (R/r)^2 outside, where
P_c = delta / (1/(2 G_out) + (1 - 2 nu_in)/(2 G_in)).  The error is the
volume-weighted L2 norm of sigma - sigma_exact over particles with r <= 0.3,
relative to that of sigma_exact; in the two-domain run the fine particles
and the coarse particles outside r = 0.15 cover the region once.
"""
from __future__ import annotations

import time

import numpy as np

E_OUT = 1e5
NU = 0.3
DELTA = 0.01
R_INC = 0.05
R_EVAL = 0.3
V_STOP = 1e-6


def contact_pressure(delta, E_out, E_in, nu_out, nu_in):
    """Interface pressure of the misfitting inclusion (compatibility condition of Sec. 4.3)."""
    G_out = E_out / (2.0 * (1.0 + nu_out))
    G_in = E_in / (2.0 * (1.0 + nu_in))
    return delta / (1.0 / (2.0 * G_out) + (1.0 - 2.0 * nu_in) / (2.0 * G_in))


def exact_stress(x, R, Pc, centre=(0.5, 0.5)):
    """Cartesian 2 x 2 stress of the plane-strain Eshelby solution at points x [n, 2]."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(centre)
    r = np.linalg.norm(d, axis=1)
    er = d / np.maximum(r, 1e-300)[:, None]
    et = np.stack([-er[:, 1], er[:, 0]], axis=1)
    ratio2 = (R / np.maximum(r, 1e-300)) ** 2
    srr = np.where(r < R, -Pc, -Pc * ratio2)
    stt = np.where(r < R, -Pc, Pc * ratio2)
    return srr[:, None, None] * er[:, :, None] * er[:, None, :] + stt[:, None, None] * et[:, :, None] * et[:, None, :]


def cauchy_stress(F, mu, lam):
    """sigma = P F^T / J of compressible Neo-Hookean material in plane strain, per particle."""
    F = np.asarray(F, dtype=np.float64)
    J = F[:, 0, 0] * F[:, 1, 1] - F[:, 0, 1] * F[:, 1, 0]
    FiT = np.empty_like(F)  # F^-T
    FiT[:, 0, 0] = F[:, 1, 1] / J
    FiT[:, 1, 1] = F[:, 0, 0] / J
    FiT[:, 0, 1] = -F[:, 1, 0] / J
    FiT[:, 1, 0] = -F[:, 0, 1] / J
    P = np.asarray(mu)[:, None, None] * (F - FiT) + (np.asarray(lam) * np.log(J))[:, None, None] * FiT
    return np.einsum("pij,pkj->pik", P, F) / J[:, None, None]


def lame(E, nu):
    E, nu = np.asarray(E, dtype=np.float64), np.asarray(nu, dtype=np.float64)
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def stress_error(parts, R, Pc, r_eval=R_EVAL):
    """Relative volume-weighted L2 stress error; parts holds (x, F, mat, vol, E, nu) per domain."""
    num = den = 0.0
    for x, F, mat, vol, E, nu in parts:
        mu, lam = lame(np.asarray(E)[mat], np.asarray(nu)[mat])
        s = cauchy_stress(F, mu, lam)
        se = exact_stress(x, R, Pc)
        w = vol * (np.linalg.norm(x - 0.5, axis=1) <= r_eval)
        num += float(np.sum(w * np.sum((s - se) ** 2, axis=(1, 2))))
        den += float(np.sum(w * np.sum(se ** 2, axis=(1, 2))))
    return float(np.sqrt(num / den))


def run(ctx, mode, ratio, inv_dx, precision, max_frames=20000, check_every=10, warm_start=False):
    """One run to static equilibrium ("single" or "dual"); returns frames, wall
    time of the frame loop (inputs already resident), particle count and the
    stress error.  warm_start applies to the dual run's Schwarz iterations."""
    import torch

    from . import binding, scenes

    dt = 0.01 * 50.0 / inv_dx
    mixed = precision == binding.OSMPM_MIXED
    so = binding.solve_opts(cg_rtol=1e-5 if mixed else 1e-10)
    kw = dict(r_inc=R_INC, E_matrix=E_OUT, E_inc=ratio * E_OUT, nu=NU, delta=DELTA, loaded=False, clamped=True)
    if mode == "single":
        sc = scenes.inclusion_single(inv_dx=inv_dx, dt=dt, **kw)
        doms = [binding.Domain(ctx, sc.B, precision=precision)]
        specs = [sc.B]

        def step():
            doms[0].single_frame(dt, so)
    else:
        sc = scenes.inclusion_scene(inv_dx_B=inv_dx // 2, inv_dx_S=inv_dx, dT=2.0 * dt, M=2, **kw)
        pair = binding.SchwarzPair(ctx, sc, precision=precision)
        doms = [pair.B, pair.S]
        specs = [sc.B, sc.S]
        opts = binding.schwarz_opts(2, eps_tol=sc.eps_tol, coarse=so, fine=so, warm_start=warm_start)

        def step():
            pair.frame(opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    frames, vmax = 0, float("inf")
    while frames < max_frames:
        step()
        frames += 1
        if frames % check_every == 0:
            vmax = max(float(torch.max(torch.abs(D.grid_state()[1]))) for D in doms)
            if vmax < V_STOP:
                break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    parts = []
    for k, (D, spec) in enumerate(zip(doms, specs)):
        x, _, _, F = D.particles_input_order()
        keep = np.ones(len(x), bool)
        if mode == "dual" and k == 0:
            keep = np.linalg.norm(spec.x - 0.5, axis=1) > 0.15
        parts.append((x[keep], F[keep], spec.mat[keep], spec.vol[keep], spec.E, spec.nu))
    Pc = contact_pressure(DELTA, E_OUT, ratio * E_OUT, NU, NU)
    out = {"mode": mode, "ratio": ratio, "inv_dx": inv_dx, "particles": int(sum(s.n_particles for s in specs)),
           "frames": frames, "converged": bool(vmax < V_STOP), "v_max": vmax, "wall_s": wall,
           "stress_L2_rel_err": stress_error(parts, R_INC, Pc)}
    if mode == "dual":
        pair.close()
    else:
        doms[0].close()
    return out
