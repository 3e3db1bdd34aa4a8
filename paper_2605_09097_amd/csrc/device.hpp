// Device-side building blocks of the OS-MPM kernels (gfx950, wave64).
//
// Grid geometry, the quadratic B-spline stencil, the compressible
// Neo-Hookean stress and its tangent, the per-particle PSD projection, and
// wave/workgroup reductions.  Arithmetic that decides an integer (the base
// node of a particle, the fixed-point node masses) is written with FMA
// contraction disabled so that it rounds exactly like the definition.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osmpm {

constexpr int kBlock = 256;  // threads per workgroup (4 waves)
constexpr int kMaxGroups = 4;

// Load of p[i] through the global address space.  Pointers copied out of a
// descriptor are generic, and a generic (flat) load also occupies the LDS
// wait counter, so a wave could not wait for its particle data without also
// draining its outstanding LDS atomics.
template <typename T>
__device__ inline T gload(const T *p, int64_t i) {
  return ((const __attribute__((address_space(1))) T *)p)[i];
}
template <typename T>
__device__ inline void gstore(T *p, int64_t i, T v) {
  ((__attribute__((address_space(1))) T *)p)[i] = v;
}
// Relaxed device-scope p[i] += v through the global address space (hardware
// floating-point atomics with -munsafe-fp-atomics).
template <typename T>
__device__ inline void gatomic_add(T *p, int64_t i, T v) {
  __hip_atomic_fetch_add((__attribute__((address_space(1))) T *)p + i, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}
// A device word that is the same for the whole launch (a flag, an index),
// read into a scalar register.
__device__ inline int uload(const int *p) { return __builtin_amdgcn_readfirstlane(gload(p, 0)); }

// Error bits raised by kernels (OR-ed into a device word).
constexpr int kErrOutOfGrid = 1;
constexpr int kErrInverted = 2;
constexpr int kErrTile = 4;

struct GridDev {
  int n[3];          // nodes per axis
  int nn;            // total nodes
  double origin[3];  // (double)origin_q * h0
  double dx, inv_dx; // (double)dx_q * h0 and 1 / dx
  long long origin_q[3];
  long long dx_q;
  double h0;
};

// Tiles of T cells (base-node positions) per axis; a tile's LDS region holds
// the (T + 2)^d nodes its particles touch.
struct TileGeom {
  int T[3], nt[3], R[3];
  int nreg, tvol, ntiles, nblocks;
};

struct SceneBC {
  int n_groups;
  int kind[kMaxGroups];
  int mask[kMaxGroups];
  double param[kMaxGroups][8];
};

template <int D, typename T = double>
struct Stencil {
  int base[D];
  T f[D];
  T w[D][3];
  T dw[D][3];
};

// Quadratic B-spline weights of a point: xi = (x - o) / dx, base =
// floor(xi - 1/2), f = xi - base.  Returns false when the 3^d stencil leaves
// the grid; the base is then clamped so every later access stays in bounds.
// The base and f are always formed in FP64 (the base decides the bin); the
// weights are evaluated in T from f rounded to T.
template <int D, typename T>
__device__ inline bool stencil_eval(const double *xp, const GridDev &g, Stencil<D, T> &s) {
#pragma clang fp contract(off)
  bool ok = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double xi = (xp[a] - g.origin[a]) * g.inv_dx;
    double bf = __builtin_floor(xi - 0.5);
    const double hi = (double)(g.n[a] - 3);
    if (!(bf >= 0.0 && bf <= hi)) {
      ok = false;
      bf = (bf > hi) ? hi : 0.0;
    }
    const T f = (T)(xi - bf);
    const T t0 = T(1.5) - f, t1 = f - T(1.0), t2 = f - T(0.5);
    const T idx = (T)g.inv_dx;
    s.base[a] = (int)bf;
    s.f[a] = f;
    s.w[a][0] = T(0.5) * (t0 * t0);
    s.w[a][1] = T(0.75) - t1 * t1;
    s.w[a][2] = T(0.5) * (t2 * t2);
    s.dw[a][0] = -t0 * idx;
    s.dw[a][1] = T(-2.0) * t1 * idx;
    s.dw[a][2] = t2 * idx;
  }
  return ok;
}

// N_ip of stencil offset k: w_x w_y in 2D, (w_x w_y) w_z in 3D (this product
// order feeds the fixed-point masses).
template <int D, typename T>
__device__ inline T stencil_N(const Stencil<D, T> &s, const int *k) {
#pragma clang fp contract(off)
  if constexpr (D == 2) {
    return s.w[0][k[0]] * s.w[1][k[1]];
  } else {
    return (s.w[0][k[0]] * s.w[1][k[1]]) * s.w[2][k[2]];
  }
}

template <int D, typename T>
__device__ inline void stencil_gradN(const Stencil<D, T> &s, const int *k, T *gN) {
  if constexpr (D == 2) {
    gN[0] = s.dw[0][k[0]] * s.w[1][k[1]];
    gN[1] = s.w[0][k[0]] * s.dw[1][k[1]];
  } else {
    gN[0] = (s.dw[0][k[0]] * s.w[1][k[1]]) * s.w[2][k[2]];
    gN[1] = (s.w[0][k[0]] * s.dw[1][k[1]]) * s.w[2][k[2]];
    gN[2] = (s.w[0][k[0]] * s.w[1][k[1]]) * s.dw[2][k[2]];
  }
}

template <int D>
constexpr int stencil_count() {
  return D == 3 ? 27 : 9;
}

template <int D>
__device__ inline void stencil_offset(int s, int *k) {
  k[0] = s % 3;
  k[1] = (s / 3) % 3;
  if constexpr (D == 3) k[2] = s / 9;
}

template <int D>
__device__ inline int node_flat(const GridDev &g, const int *idx) {
  if constexpr (D == 2) {
    return idx[0] + g.n[0] * idx[1];
  } else {
    return idx[0] + g.n[0] * (idx[1] + g.n[1] * idx[2]);
  }
}

template <int D>
__device__ inline void node_unflat(const GridDev &g, int i, int *idx) {
  idx[0] = i % g.n[0];
  if constexpr (D == 2) {
    idx[1] = i / g.n[0];
  } else {
    idx[1] = (i / g.n[0]) % g.n[1];
    idx[2] = i / (g.n[0] * g.n[1]);
  }
}

// x_i = (origin_q + i * dx_q) * h0
template <int D>
__device__ inline void node_position(const GridDev &g, const int *idx, double *x) {
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = (double)(g.origin_q[a] + (long long)idx[a] * g.dx_q) * g.h0;
}

// Fixed-point node-mass contribution rint(N * (m_p * 2^32 / m_ref)).
__device__ inline long long fixed_mass(double N, double mq) {
#pragma clang fp contract(off)
  return (long long)__builtin_rint(N * mq);
}

// ---------------------------------------------------------------- tiles
// Origin (lowest base node) of tile t, tiles numbered x fastest.
__device__ inline void tile_origin(const TileGeom &tg, int t, int *org) {
  org[0] = (t % tg.nt[0]) * tg.T[0];
  org[1] = ((t / tg.nt[0]) % tg.nt[1]) * tg.T[1];
  org[2] = (t / (tg.nt[0] * tg.nt[1])) * tg.T[2];
}

// Entry k (row-major a*D+b) of F = I + H for a particle whose stored
// displacement gradient H is in rows [k][cap].
template <int D, typename TB>
__device__ inline double load_F(const TB *H, int64_t cap, int p, int k) {
  return (double)H[k * cap + p] + ((k % (D + 1)) == 0 ? 1.0 : 0.0);
}

// ---------------------------------------------------------------- small dense algebra
template <int D, typename T>
__device__ inline T det(const T *F) {
  if constexpr (D == 2) {
    return F[0] * F[3] - F[1] * F[2];
  } else {
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
  }
}

template <int D, typename T>
__device__ inline void cofactor(const T *F, T *C) {
  if constexpr (D == 2) {
    C[0] = F[3];
    C[1] = -F[2];
    C[2] = -F[1];
    C[3] = F[0];
  } else {
    C[0] = F[4] * F[8] - F[5] * F[7];
    C[1] = F[5] * F[6] - F[3] * F[8];
    C[2] = F[3] * F[7] - F[4] * F[6];
    C[3] = F[2] * F[7] - F[1] * F[8];
    C[4] = F[0] * F[8] - F[2] * F[6];
    C[5] = F[1] * F[6] - F[0] * F[7];
    C[6] = F[1] * F[5] - F[2] * F[4];
    C[7] = F[2] * F[3] - F[0] * F[5];
    C[8] = F[0] * F[4] - F[1] * F[3];
  }
}

// Neo-Hookean first Piola stress P = mu (F - F^-T) + lam ln J F^-T and,
// optionally, A = dP/dF stored as an n x n matrix, n = D*D, index (a*D+b),
// in the arithmetic of T.
template <int D, typename T>
__device__ inline bool nh_stress(const T *F, T mu, T lam, T *P, T *A) {
  constexpr int n = D * D;
  const T J = det<D, T>(F);
  if (!(J > T(0))) return false;
  const T lnJ = log(J);
  T C[n], Fi[n];
  cofactor<D, T>(F, C);
  const T iJ = T(1) / J;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) Fi[a * D + b] = C[b * D + a] * iJ;  // F^-1
  if (P) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const T FiT = Fi[b * D + a];
        P[a * D + b] = mu * (F[a * D + b] - FiT) + lam * lnJ * FiT;
      }
  }
  if (A) {
    const T c1 = mu - lam * lnJ;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b)
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
          for (int e = 0; e < D; ++e) {
            T v = c1 * Fi[e * D + a] * Fi[b * D + c] + lam * Fi[b * D + a] * Fi[e * D + c];
            if (a == c && b == e) v += mu;
            A[(a * D + b) * n + (c * D + e)] = v;
          }
  }
  return true;
}

// True when the symmetric n x n matrix A is positive definite in T: its
// Cholesky factorisation completes with positive pivots.  Such a matrix has
// no negative eigenvalue, so its PSD projection is A itself.
template <int n, typename T>
__device__ inline bool chol_pd(const T *A) {
  T L[n * (n + 1) / 2];  // packed lower triangle, row by row
  bool ok = true;
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T v = A[i * n + j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
      if (i == j) {
        ok = ok && (v > T(0));
        L[i * (i + 1) / 2 + i] = sqrt(v > T(0) ? v : T(1));
      } else {
        L[i * (i + 1) / 2 + j] = v / L[j * (j + 1) / 2 + j];
      }
    }
  return ok;
}

// Projection of the symmetric n x n matrix A onto the PSD cone by a cyclic
// Jacobi eigendecomposition with negative eigenvalues clamped to zero.  A is
// left untouched when no eigenvalue is negative.  All indices are
// compile-time constants so W and V stay in registers.  Sweeps stop when the
// off-diagonal mass falls below the precision of T.
template <int n, typename T>
__device__ inline void psd_project(T *A) {
  constexpr T tol2 = sizeof(T) == 8 ? T(1e-32) : T(1e-13);
  T W[n * n], V[n * n];
#pragma unroll
  for (int i = 0; i < n * n; ++i) W[i] = A[i];
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? T(1) : T(0);
  T diag2 = T(0);
#pragma unroll
  for (int i = 0; i < n; ++i) diag2 += W[i * n + i] * W[i * n + i];
  for (int sweep = 0; sweep < 50; ++sweep) {
    T off = T(0);
#pragma unroll
    for (int p = 0; p < n; ++p)
#pragma unroll
      for (int q = p + 1; q < n; ++q) off += W[p * n + q] * W[p * n + q];
    if (off <= tol2 * diag2 || off == T(0)) break;
#pragma unroll
    for (int p = 0; p < n; ++p)
#pragma unroll
      for (int q = p + 1; q < n; ++q) {
        const T apq = W[p * n + q];
        if (apq != T(0)) {
          const T theta = (W[q * n + q] - W[p * n + p]) / (T(2) * apq);
          const T t = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
          const T c = T(1) / sqrt(t * t + T(1));
          const T s = t * c;
#pragma unroll
          for (int k = 0; k < n; ++k) {
            const T wkp = W[k * n + p], wkq = W[k * n + q];
            W[k * n + p] = c * wkp - s * wkq;
            W[k * n + q] = s * wkp + c * wkq;
            const T vkp = V[k * n + p], vkq = V[k * n + q];
            V[k * n + p] = c * vkp - s * vkq;
            V[k * n + q] = s * vkp + c * vkq;
          }
#pragma unroll
          for (int k = 0; k < n; ++k) {
            const T wpk = W[p * n + k], wqk = W[q * n + k];
            W[p * n + k] = c * wpk - s * wqk;
            W[q * n + k] = s * wpk + c * wqk;
          }
        }
      }
  }
  bool neg = false;
#pragma unroll
  for (int i = 0; i < n; ++i) neg |= (W[i * n + i] < T(0));
  if (!neg) return;
  T lam[n];
#pragma unroll
  for (int k = 0; k < n; ++k) lam[k] = W[k * n + k] > T(0) ? W[k * n + k] : T(0);
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < n; ++j) {
      T v = T(0);
#pragma unroll
      for (int k = 0; k < n; ++k) v += V[i * n + k] * lam[k] * V[j * n + k];
      A[i * n + j] = v;
    }
}

// Packed upper triangle of a symmetric n x n matrix: index of (r, c), r <= c.
template <int n>
__device__ __host__ constexpr int sym_index(int r, int c) {
  return r * n - (r * (r - 1)) / 2 + (c - r);
}

// Cyclic Jacobi eigendecomposition of a small symmetric m x m matrix W
// (m = 2: one rotation, exact): on return the diagonal of W holds the
// eigenvalues and the columns of Q the eigenvectors, W_in = Q diag(W) Q^T.
template <int m, typename T>
__device__ inline void jacobi_eig(T *W, T *Q) {
  constexpr T tol2 = sizeof(T) == 8 ? T(1e-32) : T(1e-13);
#pragma unroll
  for (int i = 0; i < m; ++i)
#pragma unroll
    for (int j = 0; j < m; ++j) Q[i * m + j] = (i == j) ? T(1) : T(0);
  T diag2 = T(0);
#pragma unroll
  for (int i = 0; i < m; ++i) diag2 += W[i * m + i] * W[i * m + i];
  for (int sweep = 0; sweep < (m == 2 ? 1 : 12); ++sweep) {
    T off = T(0);
#pragma unroll
    for (int p = 0; p < m; ++p)
#pragma unroll
      for (int q = p + 1; q < m; ++q) off += W[p * m + q] * W[p * m + q];
    if (off <= tol2 * diag2 || off == T(0)) break;
#pragma unroll
    for (int p = 0; p < m; ++p)
#pragma unroll
      for (int q = p + 1; q < m; ++q) {
        const T apq = W[p * m + q];
        if (apq != T(0)) {
          const T theta = (W[q * m + q] - W[p * m + p]) / (T(2) * apq);
          const T t = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
          const T c = T(1) / sqrt(t * t + T(1));
          const T s = t * c;
#pragma unroll
          for (int k = 0; k < m; ++k) {
            const T wkp = W[k * m + p], wkq = W[k * m + q];
            W[k * m + p] = c * wkp - s * wkq;
            W[k * m + q] = s * wkp + c * wkq;
            const T qkp = Q[k * m + p], qkq = Q[k * m + q];
            Q[k * m + p] = c * qkp - s * qkq;
            Q[k * m + q] = s * qkp + c * qkq;
          }
#pragma unroll
          for (int k = 0; k < m; ++k) {
            const T wpk = W[p * m + k], wqk = W[q * m + k];
            W[p * m + k] = c * wpk - s * wqk;
            W[q * m + k] = s * wpk + c * wqk;
          }
        }
      }
  }
}

// Elastoplastic extension (the paper names elastoplastic hinges as future
// work): the particle holds the elastic part F^E of F = F^E F^P; after the
// deformation-gradient update F^E is projected onto the von Mises set in
// logarithmic strain, |dev eps| <= tau_y / (2 mu), eps_k = ln s_k over the
// singular values s_k.  The closest point keeps tr eps and the principal
// directions: with F^T F = Q diag(s^2) Q^T, F <- F Q diag(exp(-delta n)) Q^T,
// n = dev eps / |dev eps|, delta = |dev eps| - tau_y / (2 mu).  Returns
// whether F changed; a material with tau_y <= 0 or infinite is elastic.
template <int D>
__device__ inline bool von_mises_project(double *F, double mu, double tau_y) {
  if (!(tau_y > 0.0) || isinf(tau_y) || !(mu > 0.0)) return false;
  double W[D * D], Q[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) t += F[k * D + a] * F[k * D + b];
      W[a * D + b] = t;
    }
  jacobi_eig<D, double>(W, Q);
  double e[D], mean = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double s2 = W[k * D + k];
    if (!(s2 > 0.0)) return false;  // singular: the solver's det check reports it
    e[k] = 0.5 * log(s2);
    mean += e[k];
  }
  mean *= 1.0 / D;
  double nrm2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    e[k] -= mean;
    nrm2 += e[k] * e[k];
  }
  const double nrm = sqrt(nrm2), ky = tau_y / (2.0 * mu);
  if (!(nrm > ky)) return false;
  const double c = (nrm - ky) / nrm;
  double f[D], S[D * D], Fo[D * D];
#pragma unroll
  for (int k = 0; k < D; ++k) f[k] = exp(-c * e[k]);
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) t += Q[a * D + k] * f[k] * Q[b * D + k];
      S[a * D + b] = t;
    }
#pragma unroll
  for (int k = 0; k < D * D; ++k) Fo[k] = F[k];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) t += Fo[a * D + k] * S[k * D + b];
      F[a * D + b] = t;
    }
  return true;
}

// Folded Neo-Hookean tangent Atil = V C^T A C (A = dP/dF at F, C: G -> G F^n,
// packed upper triangle, n = D*D) built from the analytic eigensystem of the
// Hessian of an isotropic energy (Smith, de Goes and Kim, "Analytic
// Eigensystems for Isotropic Distortion Energies", 2019), with negative
// eigenvalues clamped to zero when `project` is set: the PSD projection of A
// without forming A or running a D^2 x D^2 eigensolve.  With F = U S V^T
// (S = diag(s), from the eigendecomposition of F^T F), psi_i = dPsi/ds_i =
// mu s_i + (lam ln J - mu) / s_i, and for each pair i < j
//   twist  Q = (u_i v_j^T - u_j v_i^T) / sqrt2, eigenvalue mu + (lam ln J - mu) / (s_i s_j),
//   flip   Q = (u_i v_j^T + u_j v_i^T) / sqrt2, eigenvalue mu + (mu - lam ln J) / (s_i s_j);
// the remaining D modes are U diag(z) V^T over the eigenvectors z of the
// D x D Hessian in the singular values, H_ii = mu + (mu + lam - lam ln J) /
// s_i^2, H_ij = lam / (s_i s_j), whose clamped form replaces H (H itself
// when positive definite).  Each mode Q enters Atil as V vec(Q F^nT)
// vec(Q F^nT)^T times its (clamped) eigenvalue.
template <int D, typename T>
__device__ inline void nh_folded_tangent(const T *F, const T *Fn, T mu, T lam, T Vol, bool project, T *At) {
  constexpr int n = D * D;
  constexpr int ns = n * (n + 1) / 2;
  T W[D * D], Vv[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T c = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) c += F[k * D + a] * F[k * D + b];
      W[a * D + b] = c;
    }
  jacobi_eig<D, T>(W, Vv);
  T sg[D], isg[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T e = W[i * D + i];
    sg[i] = sqrt(e > T(0) ? e : T(0));
    isg[i] = sg[i] > T(0) ? T(1) / sg[i] : T(0);
  }
  const T lnJ = log(det<D, T>(F));
  // U = F V S^-1 and g_j = F^n v_j, both column-major by mode: U[a*D+i] = (u_i)_a
  T U[D * D], g[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T fu = T(0), fg = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        fu += F[a * D + k] * Vv[k * D + i];
        fg += Fn[a * D + k] * Vv[k * D + i];
      }
      U[a * D + i] = fu * isg[i];
      g[a * D + i] = fg;
    }
#pragma unroll
  for (int k = 0; k < ns; ++k) At[k] = T(0);
  const T c0 = lam * lnJ - mu;
  const T rs2 = T(0.70710678118654752440);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i + 1; j < D; ++j) {
      const T iss = isg[i] * isg[j];
      T lt = mu + c0 * iss, lf = mu - c0 * iss;
      if (project) {
        lt = lt > T(0) ? lt : T(0);
        lf = lf > T(0) ? lf : T(0);
      }
      T wt[n], wf[n];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          const T x = U[a * D + i] * g[b * D + j], y = U[a * D + j] * g[b * D + i];
          wt[a * D + b] = rs2 * (x - y);
          wf[a * D + b] = rs2 * (x + y);
        }
#pragma unroll
      for (int r = 0; r < n; ++r)
#pragma unroll
        for (int c = r; c < n; ++c) At[sym_index<n>(r, c)] += lt * wt[r] * wt[c] + lf * wf[r] * wf[c];
    }
  // scaling block
  T H[D * D];
  const T cd = mu + lam - lam * lnJ;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) H[i * D + j] = (i == j) ? mu + cd * isg[i] * isg[i] : lam * isg[i] * isg[j];
  if (project && !chol_pd<D, T>(H)) {
    T Z[D * D];
    jacobi_eig<D, T>(H, Z);
    T h[D];
#pragma unroll
    for (int k = 0; k < D; ++k) h[k] = H[k * D + k] > T(0) ? H[k * D + k] : T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T v = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) v += Z[i * D + k] * h[k] * Z[j * D + k];
        H[i * D + j] = v;
      }
  }
  // Atil += sum_ij H_ij s_i s_j^T with s_i = vec(u_i g_i^T), one i at a time
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T si[n], ti[n];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        si[a * D + b] = U[a * D + i] * g[b * D + i];
        T tv = T(0);
#pragma unroll
        for (int j = 0; j < D; ++j) tv += H[i * D + j] * U[a * D + j] * g[b * D + j];
        ti[a * D + b] = tv;
      }
#pragma unroll
    for (int r = 0; r < n; ++r)
#pragma unroll
      for (int c = r; c < n; ++c) At[sym_index<n>(r, c)] += si[r] * ti[c];
  }
#pragma unroll
  for (int k = 0; k < ns; ++k) At[k] *= Vol;
}


// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a workgroup of kBlock threads; every thread gets the total.
__device__ inline double block_sum(double v, double *lds4) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) lds4[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) t += lds4[i];
  return t;
}

// Sum of a partials array in a fixed order (deterministic), computed by one
// workgroup; every thread gets the total.
__device__ inline double reduce_partials(const double *part, int n, double *lds4) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) v += part[i];
  return block_sum(v, lds4);
}

}  // namespace osmpm
