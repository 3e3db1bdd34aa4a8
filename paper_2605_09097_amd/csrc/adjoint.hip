// Reverse-mode kernels of the OS-MPM frame: transposes of P2G, G2P, the
// projection Pi_{S->B}, the interpolation I_{B->S} and T_m, and the
// right-hand side and input terms of the adjoint of an implicit solve (the
// adjoint linear system itself runs on the forward CG kernels).
//
// Particle adjoints are FP64, component-major [component][n] and indexed by
// particle id (the particle's position in the input arrays), so the sorts
// between steps need no permutation: a kernel that walks a stored state in
// its sorted order reads and writes the adjoint at the particle's id.
// Grid adjoints are FP64 [node][d].  Arithmetic is FP64 in both paths; the
// stored forward states are read in their bulk type.
#include "kernels.hpp"

namespace osmpm {

// d2 N_ip / dx_p dx_p (symmetric d x d) at stencil offset k; per axis the
// second derivative of the quadratic B-spline is (1, -2, 1) / dx^2 for the
// three offsets.
template <int D>
__device__ inline void stencil_hess(const Stencil<D> &st, const int *k, double inv_dx, double *Hs) {
  double w[3] = {1.0, 1.0, 1.0}, dw[3] = {0.0, 0.0, 0.0}, ddw[3] = {0.0, 0.0, 0.0};
  const double i2 = inv_dx * inv_dx;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    w[a] = st.w[a][k[a]];
    dw[a] = st.dw[a][k[a]];
    ddw[a] = (k[a] == 1 ? -2.0 : 1.0) * i2;
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double v = 1.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        if (a == b)
          v *= (c == a) ? ddw[c] : w[c];
        else
          v *= (c == a || c == b) ? dw[c] : w[c];
      }
      Hs[a * D + b] = v;
    }
}

// ---------------------------------------------------------------- P2G transposed
// Given mbar, vnbar on the nodes (adjoints of the node mass and of
// v = (mv)/m), adds to the particle adjoints of x, v, B:
//   vbar += m_p N pb,  Bbar += m_p N Dinv pb (x_i - x_p)^T,
//   xbar += m_p [(mt + pb.w) grad N - N Dinv B^T pb],
// pb = vnbar_i / m_i, mt = mbar_i - vnbar_i.v_i / m_i, w = v_p + Dinv B_p (x_i - x_p).
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_adj_p2g(GridDev g, int np, int64_t cap, const double *x, const TB *v, const TB *B,
                          const double *mass, const int *id, const double *m, const double *vn, const double *mbar,
                          const double *vnbar, double *ax, double *av, double *aB) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const double Dinv = 4.0 * g.inv_dx * g.inv_dx;
  double xp[D], vp[D], Bp[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xp[a] = x[a * cap + p];
    vp[a] = (double)v[a * cap + p];
  }
#pragma unroll
  for (int k = 0; k < D * D; ++k) Bp[k] = (double)B[k * cap + p];
  Stencil<D> st;
  stencil_eval<D>(xp, g, st);
  const double mp = mass[p];
  const int q = id[p];
  double gx[D], gv[D], gB[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    gx[a] = 0.0;
    gv[a] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < D * D; ++k) gB[k] = 0.0;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int i = node_flat<D>(g, idx);
    const double N = stencil_N<D>(st, k);
    double gN[D], dxv[D];
    stencil_gradN<D>(st, k, gN);
#pragma unroll
    for (int a = 0; a < D; ++a) dxv[a] = ((double)k[a] - st.f[a]) * g.dx;
    const double mi = m[i];
    double pb[D], mt = mbar[i];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      pb[a] = 0.0;
      if (mi > 0.0) {
        pb[a] = vnbar[i * D + a] / mi;
        mt -= vnbar[i * D + a] * vn[i * D + a] / mi;
      }
    }
    double pw = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double aff = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) aff += Bp[a * D + b] * dxv[b];
      pw += pb[a] * (vp[a] + Dinv * aff);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      gv[a] += mp * N * pb[a];
#pragma unroll
      for (int b = 0; b < D; ++b) gB[a * D + b] += mp * N * Dinv * pb[a] * dxv[b];
      double bt = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) bt += Bp[b * D + a] * pb[b];
      gx[a] += mp * ((mt + pw) * gN[a] - N * Dinv * bt);
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    ax[a * (int64_t)np + q] += gx[a];
    av[a * (int64_t)np + q] += gv[a];
  }
#pragma unroll
  for (int k = 0; k < D * D; ++k) aB[k * (int64_t)np + q] += gB[k];
}

// ---------------------------------------------------------------- G2P transposed
// The stored state before G2P (x, F), the grid displacement u and the active
// nodes (m > 0); (ix, iv, iB, iF) is the adjoint of the state after G2P.
// Adds ubar on the nodes (FP64 atomics) and the adjoint of x and F before
// G2P: xbar += ix + sum_i [(u_i.vt + u_i.(iB dx_i))/dt grad N - N iB^T u_i/dt
// + Hs_i (F iF^T u_i)], Fbar += (I + G_u)^T iF, vt = iv + dt ix.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_adj_g2p(GridDev g, int np, int64_t cap, const double *x, const TB *F, const int *id,
                          const double *m, const double *u, double dt, const double *ix, const double *iv,
                          const double *iB, const double *iF, double *ubar, double *ox, double *oF) {
  constexpr int n = D * D;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int q = id[p];
  double xp[D], Fp[n], Fb[n], Bb[n], vt[D], gx[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xp[a] = x[a * cap + p];
    vt[a] = iv[a * (int64_t)np + q] + dt * ix[a * (int64_t)np + q];
    gx[a] = ix[a * (int64_t)np + q];
  }
#pragma unroll
  for (int k = 0; k < n; ++k) {
    Fp[k] = load_F<D>(F, cap, p, k);
    Fb[k] = iF[k * (int64_t)np + q];
    Bb[k] = iB[k * (int64_t)np + q];
  }
  double M1[n], M2[n];  // iF F^T, F iF^T
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double t1 = 0.0, t2 = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        t1 += Fb[a * D + c] * Fp[b * D + c];
        t2 += Fp[a * D + c] * Fb[b * D + c];
      }
      M1[a * D + b] = t1;
      M2[a * D + b] = t2;
    }
  Stencil<D> st;
  stencil_eval<D>(xp, g, st);
  double G[n];
#pragma unroll
  for (int k = 0; k < n; ++k) G[k] = 0.0;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int i = node_flat<D>(g, idx);
    if (!(m[i] > 0.0)) continue;
    const double N = stencil_N<D>(st, k);
    double gN[D], dxv[D], Hs[n], ui[D];
    stencil_gradN<D>(st, k, gN);
    stencil_hess<D>(st, k, g.inv_dx, Hs);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      dxv[a] = ((double)k[a] - st.f[a]) * g.dx;
      ui[a] = u[i * D + a];
    }
    double Bx[D], Btu[D], Mu[D], uv = 0.0, uBx = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double t = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        t += Bb[a * D + b] * dxv[b];
        t2 += Bb[b * D + a] * ui[b];
        t3 += M2[a * D + b] * ui[b];
      }
      Bx[a] = t;
      Btu[a] = t2;
      Mu[a] = t3;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      uv += ui[a] * vt[a];
      uBx += ui[a] * Bx[a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) t += M1[a * D + b] * gN[b];
      atomicAdd(&ubar[i * D + a], N * vt[a] / dt + N * Bx[a] / dt + t);
      double h = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) h += Hs[a * D + b] * Mu[b];
      gx[a] += (uv + uBx) / dt * gN[a] - N * Btu[a] / dt + h;
#pragma unroll
      for (int b = 0; b < D; ++b) G[a * D + b] += ui[a] * gN[b];
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) ox[a * (int64_t)np + q] += gx[a];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double t = Fb[a * D + b];
#pragma unroll
      for (int c = 0; c < D; ++c) t += G[c * D + a] * Fb[c * D + b];
      oF[(a * D + b) * (int64_t)np + q] += t;
    }
}

// ---------------------------------------------------------------- implicit solve
// Right-hand side of the adjoint system H_ff lambda = ubar_f: the CG start
// kernel forms r_0 = -g, so g = -ubar on the free DOFs (the free mask comes
// from the Dirichlet setup of the same solve).  Moves the domain to the CG
// start phase.
__global__ void __launch_bounds__(kBlock) k_adj_set_rhs(const DomDesc *dd, const double *ubar) {
  const DomDesc &dm = dd[blockIdx.y];
  const int nb = node_blocks(dm.ndof);
  if (!*dm.active || (int)blockIdx.x >= nb) return;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < dm.ndof; k += nb * kBlock)
    dm.gg[k] = dm.fr[k] ? -ubar[k] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) dm.ss->phase = kPhaseCgInit;
}

// y = sum_p V (A : dF(lambda)) c_ip through the particles (the stiffness part
// of H lambda; lambda vanishes on the Dirichlet DOFs, so the lumped-mass part
// does not reach them).  Tangents Atil in the packed folded form.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_adj_hvp(const DomDesc *dd, const TB *lam, double *y) {
  constexpr int n = D * D;
  constexpr int ns = n * (n + 1) / 2;
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= dm.np) return;
  const GridDev &g = dm.g;
  const int64_t cap = dm.cap;
  const double *x = dm.pb[*dm.cur].x;
  const TB *Atil = static_cast<const TB *>(dm.Atil);
  double xp[D];
#pragma unroll
  for (int a = 0; a < D; ++a) xp[a] = x[a * cap + p];
  Stencil<D> st;
  stencil_eval<D>(xp, g, st);
  double G[n];
#pragma unroll
  for (int k = 0; k < n; ++k) G[k] = 0.0;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int i = node_flat<D>(g, idx);
    double gN[D];
    stencil_gradN<D>(st, k, gN);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) G[a * D + b] += (double)lam[i * D + a] * gN[b];
  }
  double T[n];
#pragma unroll
  for (int r = 0; r < n; ++r) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < n; ++c)
      t += (double)((r <= c) ? Atil[sym_index<n>(r, c) * cap + p] : Atil[sym_index<n>(c, r) * cap + p]) * G[c];
    T[r] = t;
  }
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int i = node_flat<D>(g, idx);
    double gN[D];
    stencil_gradN<D>(st, k, gN);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) t += T[a * D + b] * gN[b];
      atomicAdd(&y[i * D + a], t);
    }
  }
}

// Node inputs of the solve: on free DOFs vnbar += lambda m / dt and
// mbar -= lambda . ((u - dt v) / dt^2 - g); on Schwarz receiver DOFs
// (Dirichlet, not scene-constrained) the data receive
// vbcbar += dt (ubar - (H lambda)).
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_adj_solve_nodes(const DomDesc *dd, double dt, double gx, double gy, double gz, const double *ubar,
                                  const double *hl, int use_schwarz, double *mbar, double *vnbar, double *vbcbar) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= dm.g.nn) return;
  const double m = dm.m[i];
  if (!(m > 0.0)) return;
  const TB *lam = static_cast<const TB *>(dm.del);
  const double grav[3] = {gx, gy, gz};
  double mb = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int k = i * D + a;
    if (dm.fr[k]) {
      const double l = (double)lam[k];
      vnbar[k] += l * m / dt;
      mb -= l * ((dm.u[k] - dt * dm.vn[k]) / (dt * dt) - grav[a]);
    } else if (vbcbar && use_schwarz && dm.bcg[k] < 0 && dm.recv[i]) {
      vbcbar[k] += dt * (ubar[k] - hl[k]);
    }
  }
  mbar[i] += mb;
}

// Particle inputs of the solve: phi_p = V P(F(u)) : (G_lambda F^n) with
// F(u) = (I + G_u) F^n.  Adds Fbar -= V ((I + G_u)^T (A : L) + G_lambda^T P),
// xbar -= V sum_i Hs_i ((A:L) F^nT)^T u_i + (P F^nT)^T lambda_i), and the
// material adjoints mubar -= V (F - F^-T) : L, lambar -= V ln J F^-T : L,
// L = G_lambda F^n, with the exact (unprojected) tangent A.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_adj_solve_particles(const DomDesc *dd, double *ax, double *aF, int np_adj, double *mubar,
                                      double *lambar) {
  constexpr int n = D * D;
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  __shared__ double smu[64], sla[64];
  for (int k = threadIdx.x; k < 64; k += blockDim.x) {
    smu[k] = 0.0;
    sla[k] = 0.0;
  }
  __syncthreads();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < dm.np) {
    const GridDev &g = dm.g;
    const int64_t cap = dm.cap;
    const PartPtrs &P0 = dm.pb[*dm.cur];
    const TB *Fv = static_cast<const TB *>(P0.F);
    const TB *lam = static_cast<const TB *>(dm.del);
    const int q = P0.id[p];
    double xp[D], Fn[n], Gu[n], Gl[n];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = P0.x[a * cap + p];
#pragma unroll
    for (int k = 0; k < n; ++k) {
      Fn[k] = load_F<D>(Fv, cap, p, k);
      Gu[k] = 0.0;
      Gl[k] = 0.0;
    }
    Stencil<D> st;
    stencil_eval<D>(xp, g, st);
#pragma unroll
    for (int s = 0; s < stencil_count<D>(); ++s) {
      int k[3], idx[3];
      stencil_offset<D>(s, k);
#pragma unroll
      for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
      const int i = node_flat<D>(g, idx);
      double gN[D];
      stencil_gradN<D>(st, k, gN);
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          Gu[a * D + b] += dm.u[i * D + a] * gN[b];
          Gl[a * D + b] += (double)lam[i * D + a] * gN[b];
        }
    }
    double H[n], F[n], L[n];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) H[a * D + b] = (a == b ? 1.0 : 0.0) + Gu[a * D + b];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        double t = 0.0, t2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          t += H[a * D + c] * Fn[c * D + b];
          t2 += Gl[a * D + c] * Fn[c * D + b];
        }
        F[a * D + b] = t;
        L[a * D + b] = t2;
      }
    const int mt = P0.mat[p];
    const double mu = dm.mu[mt], la = dm.lam[mt], V = P0.vol[p];
    double Pk[n], A[n * n];
    if (nh_stress<D, double>(F, mu, la, Pk, A)) {
      const double J = det<D, double>(F), lnJ = log(J);
      double C[n];
      cofactor<D, double>(F, C);
      double smu_p = 0.0, sla_p = 0.0;
#pragma unroll
      for (int k = 0; k < n; ++k) {
        smu_p += (F[k] - C[k] / J) * L[k];
        sla_p += lnJ * C[k] / J * L[k];
      }
      if (mt < 64) {
        atomicAdd(&smu[mt], -V * smu_p);
        atomicAdd(&sla[mt], -V * sla_p);
      }
      double AL[n];
#pragma unroll
      for (int r = 0; r < n; ++r) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < n; ++c) t += A[r * n + c] * L[c];
        AL[r] = t;
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          double t = 0.0;
#pragma unroll
          for (int c = 0; c < D; ++c) t += H[c * D + a] * AL[c * D + b] + Gl[c * D + a] * Pk[c * D + b];
          aF[(a * D + b) * (int64_t)np_adj + q] -= V * t;
        }
      double Y1[n], Y2[n];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          double t1 = 0.0, t2 = 0.0;
#pragma unroll
          for (int c = 0; c < D; ++c) {
            t1 += AL[a * D + c] * Fn[b * D + c];
            t2 += Pk[a * D + c] * Fn[b * D + c];
          }
          Y1[a * D + b] = t1;
          Y2[a * D + b] = t2;
        }
      double gx[D];
#pragma unroll
      for (int a = 0; a < D; ++a) gx[a] = 0.0;
#pragma unroll
      for (int s = 0; s < stencil_count<D>(); ++s) {
        int k[3], idx[3];
        stencil_offset<D>(s, k);
#pragma unroll
        for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
        const int i = node_flat<D>(g, idx);
        double Hs[n], y[D];
        stencil_hess<D>(st, k, g.inv_dx, Hs);
#pragma unroll
        for (int b = 0; b < D; ++b) {
          double t = 0.0;
#pragma unroll
          for (int a = 0; a < D; ++a) t += Y1[a * D + b] * dm.u[i * D + a] + Y2[a * D + b] * (double)lam[i * D + a];
          y[b] = t;
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double t = 0.0;
#pragma unroll
          for (int b = 0; b < D; ++b) t += Hs[a * D + b] * y[b];
          gx[a] += t;
        }
      }
#pragma unroll
      for (int a = 0; a < D; ++a) ax[a * (int64_t)np_adj + q] -= V * gx[a];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 64; k += blockDim.x) {
    if (smu[k] != 0.0) atomicAdd(&mubar[k], smu[k]);
    if (sla[k] != 0.0) atomicAdd(&lambar[k], sla[k]);
  }
}

// ---------------------------------------------------------------- interface transposed
// Pi_{S->B} transposed, per active fine node j (gather over its coarse
// stencil): with num, den the projection sums of the same fine grid,
//   vnbar_j += m_j N_Ij numbar_I,  mbar_j += N_Ij (v_j.numbar_I + denbar_I),
// numbar = pbar / (den + eps), denbar = -(pbar.num) / (den + eps)^2, on the
// coarse receivers.
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_project(GridDev gB, GridDev gS, const double *mS, const double *vnS, const uint8_t *recvB,
                              const double *num, const double *den, double eps_tol, const double *pbar,
                              double *mbarS, double *vnbarS) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= gS.nn) return;
  const double m = mS[j];
  if (!(m > 0.0)) return;
  int jS[3];
  double xj[D];
  node_unflat<D>(gS, j, jS);
  node_position<D>(gS, jS, xj);
  Stencil<D> st;
  if (!stencil_eval<D>(xj, gB, st)) return;
  double vb[D], mb = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) vb[a] = 0.0;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int I = node_flat<D>(gB, idx);
    if (!recvB[I]) continue;
    const double N = stencil_N<D>(st, k);
    const double de = den[I] + eps_tol;
    double pn = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) pn += pbar[I * D + a] * num[I * D + a];
    const double denbar = -pn / (de * de);
    double vnum = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double numbar = pbar[I * D + a] / de;
      vb[a] += m * N * numbar;
      vnum += vnS[j * D + a] * numbar;
    }
    mb += N * (vnum + denbar);
  }
#pragma unroll
  for (int a = 0; a < D; ++a) vnbarS[j * D + a] += vb[a];
  mbarS[j] += mb;
}

// I_{B->S} transposed: every fine receiver scatters N_I(x_j) ibar_j to its
// active coarse stencil nodes.
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_interp(GridDev gB, GridDev gS, const double *mB, const uint8_t *recvS, const double *ibar,
                             double *vBbar) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= gS.nn || !recvS[j]) return;
  int jS[3];
  double xj[D];
  node_unflat<D>(gS, j, jS);
  node_position<D>(gS, jS, xj);
  Stencil<D> st;
  if (!stencil_eval<D>(xj, gB, st)) return;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int I = node_flat<D>(gB, idx);
    if (!(mB[I] > 0.0)) continue;
    const double N = stencil_N<D>(st, k);
#pragma unroll
    for (int a = 0; a < D; ++a) atomicAdd(&vBbar[I * D + a], N * ibar[j * D + a]);
  }
}

// T_m transposed: a += (1 - am) vbcbar, b += am vbcbar.
__global__ void __launch_bounds__(kBlock) k_adj_temporal(int64_t n, double am, const double *vbcbar, double *a, double *b) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    a[k] += (1.0 - am) * vbcbar[k];
    b[k] += am * vbcbar[k];
  }
}

// v_B = u_B / dT on the active nodes, transposed: ubar += vbar / dT.
template <int D>
__global__ void __launch_bounds__(kBlock) k_adj_vel(int nn, const double *m, const double *vbar, double dT, double *ubar) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn || !(m[i] > 0.0)) return;
#pragma unroll
  for (int a = 0; a < D; ++a) ubar[i * D + a] += vbar[i * D + a] / dT;
}

#define OSMPM_ADJ_INST_D(D)                                                                                   \
  template __global__ void k_adj_project<D>(GridDev, GridDev, const double *, const double *, const uint8_t *, \
                                            const double *, const double *, double, const double *, double *,  \
                                            double *);                                                         \
  template __global__ void k_adj_interp<D>(GridDev, GridDev, const double *, const uint8_t *, const double *,  \
                                           double *);                                                          \
  template __global__ void k_adj_vel<D>(int, const double *, const double *, double, double *);

#define OSMPM_ADJ_INST_DT(D, TB)                                                                               \
  template __global__ void k_adj_p2g<D, TB>(GridDev, int, int64_t, const double *, const TB *, const TB *,      \
                                            const double *, const int *, const double *, const double *,        \
                                            const double *, const double *, double *, double *, double *);      \
  template __global__ void k_adj_g2p<D, TB>(GridDev, int, int64_t, const double *, const TB *, const int *,     \
                                            const double *, const double *, double, const double *,             \
                                            const double *, const double *, const double *, double *, double *, \
                                            double *);                                                          \
  template __global__ void k_adj_hvp<D, TB>(const DomDesc *, const TB *, double *);                             \
  template __global__ void k_adj_solve_nodes<D, TB>(const DomDesc *, double, double, double, double,             \
                                                    const double *, const double *, int, double *, double *,     \
                                                    double *);                                                  \
  template __global__ void k_adj_solve_particles<D, TB>(const DomDesc *, double *, double *, int, double *,      \
                                                        double *);

OSMPM_ADJ_INST_D(2)
OSMPM_ADJ_INST_D(3)
OSMPM_ADJ_INST_DT(2, double)
OSMPM_ADJ_INST_DT(2, float)
OSMPM_ADJ_INST_DT(3, double)
OSMPM_ADJ_INST_DT(3, float)

}  // namespace osmpm

namespace osmpm {
// y += a x (grid-stride).
__global__ void __launch_bounds__(kBlock) k_axpy_d(int64_t n, double a, const double *x, double *y) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    y[k] += a * x[k];
}

// out[0] = sum_k x[k]^2 by one workgroup in a fixed order (strided partial
// sums per thread, then a tree over the workgroup), so the result does not
// depend on scheduling.
__global__ void __launch_bounds__(kBlock) k_sumsq_d(int64_t n, const double *x, double *out) {
  __shared__ double part[kBlock];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += kBlock) acc += x[k] * x[k];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}
}  // namespace osmpm
