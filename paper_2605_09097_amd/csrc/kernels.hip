// OS-MPM kernels for gfx950 (wave64, 256-thread workgroups).
//
// Particle-to-grid style kernels (P2G, gradient/Hessian build, CG
// Hessian-vector product) run one workgroup per tile of cells: the particles
// of a tile are contiguous after the binning sort, their 3^d stencils touch
// the (T+2)^d nodes of the tile region, which is staged in LDS (gathers) and
// accumulated in LDS with LDS atomics (scatters) before one pass of global
// atomics per node.  Node kernels are grid-stride loops over DOFs.
// Reductions go through per-workgroup partials that the consumer sums in a
// fixed order, so every scalar is deterministic run to run.
#include "kernels.hpp"

namespace osmpm {

// ====================================================================== misc
template <typename T>
__global__ void k_fill(int64_t n, T v, T *a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
template __global__ void k_fill<double>(int64_t, double, double *);
template __global__ void k_fill<float>(int64_t, float, float *);
__global__ void k_fill_i64(int64_t n, long long *a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}
__global__ void k_fill_i32(int64_t n, int v, int *a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
__global__ void k_fill_u8(int64_t n, uint8_t *a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

// [n][c] (caller layout, FP64) -> [c][cap] (library layout, storage type T)
template <typename T>
__global__ void k_aos_to_soa(int64_t n, int c, const double *src, T *dst, int64_t cap) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * c; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / c, r = i % c;
    dst[r * cap + p] = (T)src[i];
  }
}
template <typename T>
__global__ void k_soa_to_aos(int64_t n, int c, const T *src, int64_t cap, double *dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * c; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / c, r = i % c;
    dst[i] = (double)src[r * cap + p];
  }
}
template __global__ void k_aos_to_soa<double>(int64_t, int, const double *, double *, int64_t);
template __global__ void k_aos_to_soa<float>(int64_t, int, const double *, float *, int64_t);
template __global__ void k_soa_to_aos<double>(int64_t, int, const double *, int64_t, double *);
template __global__ void k_soa_to_aos<float>(int64_t, int, const float *, int64_t, double *);
__global__ void k_iota(int n, int *a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = i;
}

// ====================================================================== sort
// Tile-major bin key of the particle's base node, and the bin histogram.
template <int D>
__global__ void k_keys(int n, const double *x, int64_t cap, GridDev g, TileGeom tg, int *key, int *count,
                       int *err) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double xp[D];
#pragma unroll
  for (int a = 0; a < D; ++a) xp[a] = x[a * cap + p];
  Stencil<D> st;
  if (!stencil_eval<D>(xp, g, st)) atomicOr(err, kErrOutOfGrid);
  int t[3] = {0, 0, 0}, l[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    t[a] = st.base[a] / tg.T[a];
    l[a] = st.base[a] % tg.T[a];
  }
  const int tf = t[0] + tg.nt[0] * (t[1] + tg.nt[1] * t[2]);
  const int lf = l[0] + tg.T[0] * (l[1] + tg.T[1] * l[2]);
  const int k = tf * tg.tvol + lf;
  key[p] = k;
  atomicAdd(&count[k], 1);
}

// Exclusive scan of nk counts by one workgroup of 1024 threads, 4096
// elements per pass (each thread four consecutive counts, so loads and
// stores are coalesced); cell_start[nk] is the total.  cursor receives a copy
// of the offsets for the scatter.
__global__ void __launch_bounds__(1024) k_scan(int nk, const int *count, int *cell_start, int *cursor) {
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int carry = 0;
  for (int base = 0; base < nk; base += 4096) {
    int v[4];
    int s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int idx = base + 4 * tid + j;
      v[j] = (idx < nk) ? count[idx] : 0;
      s += v[j];
    }
    int xs = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(xs, off, 64);
      if (lane >= off) xs += y;
    }
    if (lane == 63) wsum[w] = xs;
    __syncthreads();
    if (w == 0) {
      int ws = (lane < 16) ? wsum[lane] : 0;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const int y = __shfl_up(ws, off, 64);
        if (lane >= off) ws += y;
      }
      if (lane < 16) wsum[lane] = ws;
    }
    __syncthreads();
    int excl = carry + (w > 0 ? wsum[w - 1] : 0) + (xs - s);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int idx = base + 4 * tid + j;
      if (idx < nk) {
        cell_start[idx] = excl;
        cursor[idx] = excl;
      }
      excl += v[j];
    }
    carry += wsum[15];
    __syncthreads();
  }
  if (tid == 0) cell_start[nk] = carry;
}

__global__ void k_scatter(int n, const int *key, int *cursor, int *perm) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  perm[atomicAdd(&cursor[key[p]], 1)] = p;
}

// The scatter fills each bin in arbitrary order; sorting every bin by the
// original index makes the result the stable counting sort.
__global__ void k_cellsort(int nk, const int *cell_start, int *perm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  const int s = cell_start[k], e = cell_start[k + 1];
  for (int i = s + 1; i < e; ++i) {
    const int v = perm[i];
    int j = i - 1;
    while (j >= s && perm[j] > v) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
}

template <typename T>
__global__ void k_gather(int n, int rows, const int *perm, const T *src, T *dst, int64_t cap) {
  const int64_t total = (int64_t)n * rows;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n, p = i % n;
    dst[r * cap + p] = src[r * cap + perm[p]];
  }
}
template __global__ void k_gather<double>(int, int, const int *, const double *, double *, int64_t);
template __global__ void k_gather<float>(int, int, const int *, const float *, float *, int64_t);
template __global__ void k_gather<int>(int, int, const int *, const int *, int *, int64_t);
template __global__ void k_gather<uint8_t>(int, int, const int *, const uint8_t *, uint8_t *, int64_t);

// ====================================================================== tiles
// Particle range of tile t and its node-region origin.  Returns false for
// padding blocks.
__device__ inline bool tile_range(const TileGeom &tg, const int *cell_start, int t, int &p0, int &p1, int *org) {
  if (t >= tg.ntiles) return false;
  p0 = cell_start[t * tg.tvol];
  p1 = cell_start[(t + 1) * tg.tvol];
  tile_origin(tg, t, org);
  return true;
}

// Global node of LDS region slot r (x fastest), or -1 when outside the grid.
template <int D>
__device__ inline int region_node(const TileGeom &tg, const GridDev &g, const int *org, int r) {
  int idx[3];
  idx[0] = org[0] + r % tg.R[0];
  idx[1] = org[1] + (r / tg.R[0]) % tg.R[1];
  idx[2] = (D == 3) ? org[2] + r / (tg.R[0] * tg.R[1]) : 0;
#pragma unroll
  for (int a = 0; a < D; ++a)
    if (idx[a] >= g.n[a]) return -1;
  return node_flat<D>(g, idx);
}

// Local offsets of a particle's base node in its tile; false if it does not
// belong to the tile (a corrupted binning; the particle is then skipped).
template <int D>
__device__ inline bool local_base(const TileGeom &tg, const Stencil<D> &st, const int *org, int *l) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    l[a] = st.base[a] - org[a];
    ok &= (l[a] >= 0 && l[a] < tg.T[a]);
  }
  return ok;
}

template <int D>
__device__ inline int region_slot(const TileGeom &tg, const int *l, const int *k) {
  if constexpr (D == 2) {
    return (l[0] + k[0]) + tg.R[0] * (l[1] + k[1]);
  } else {
    return (l[0] + k[0]) + tg.R[0] * ((l[1] + k[1]) + tg.R[1] * (l[2] + k[2]));
  }
}

// ====================================================================== P2G
// APIC P2G (Eq. p2g_transfer) of one tile into LDS, then global atomics.
// Also the fixed-point node masses (all particles, and per scene group).
// TB is the storage type of the particle velocity and affine matrix (FP32 in
// the mixed path).  Tile sums are accumulated in FP64 LDS (ds_add_f64, which
// measures about twice as fast as ds_add_f32 on gfx950) and added to the FP64
// grid.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_p2g(TileGeom tg, GridDev g, const int *cell_start, const double *x,
                                                const TB *v, const TB *B, const double *mass,
                                                const uint8_t *flags, int64_t cap, int n_groups, double scale,
                                                double Dinv, int want_q, double *gm, double *gmv,
                                                long long *q_all, long long *qg, int *err) {
  extern __shared__ double lds[];
  const int t = tile_of_block(tg, blockIdx.x);
  int p0, p1, org[3];
  if (!tile_range(tg, cell_start, t, p0, p1, org) || p0 == p1) return;
  const int nreg = tg.nreg;
  long long *lq = reinterpret_cast<long long *>(lds);
  double *lm = reinterpret_cast<double *>(lq + (size_t)(1 + kMaxGroups) * nreg);
  double *lmv = lm + nreg;
  const int nq = want_q ? 1 + n_groups : 0;
  for (int r = threadIdx.x; r < nreg * (1 + D); r += kBlock) lm[r] = 0.0;
  for (int r = threadIdx.x; r < nreg * nq; r += kBlock) lq[r] = 0;
  __syncthreads();
  for (int p = p0 + threadIdx.x; p < p1; p += kBlock) {
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
    int l[3];
    if (!local_base<D>(tg, st, org, l)) {
      atomicOr(err, kErrTile);
      continue;
    }
    const double mp = mass[p];
    const double mq = mp * scale;
    const uint8_t fl = flags[p];
#pragma unroll
    for (int s = 0; s < stencil_count<D>(); ++s) {
      int k[3];
      stencil_offset<D>(s, k);
      const double N = stencil_N<D>(st, k);
      double dxv[D];
#pragma unroll
      for (int a = 0; a < D; ++a) dxv[a] = ((double)k[a] - st.f[a]) * g.dx;
      const int r = region_slot<D>(tg, l, k);
      const double mN = mp * N;
      atomicAdd(&lm[r], (double)(TB)mN);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double aff = 0.0;
#pragma unroll
        for (int b = 0; b < D; ++b) aff += Bp[a * D + b] * dxv[b];
        atomicAdd(&lmv[a * nreg + r], (double)(TB)(mN * (vp[a] + Dinv * aff)));
      }
      if (want_q) {
        const long long q = fixed_mass(N, mq);
        atomicAdd(reinterpret_cast<unsigned long long *>(&lq[r]), (unsigned long long)q);
        for (int gi = 0; gi < n_groups; ++gi)
          if (fl & (2u << gi))
            atomicAdd(reinterpret_cast<unsigned long long *>(&lq[(1 + gi) * nreg + r]), (unsigned long long)q);
      }
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < nreg; r += kBlock) {
    const int i = region_node<D>(tg, g, org, r);
    if (i < 0) continue;
    const double m = lm[r];
    if (m != 0.0) {
      atomicAdd(&gm[i], m);
#pragma unroll
      for (int a = 0; a < D; ++a) atomicAdd(&gmv[i * D + a], lmv[a * nreg + r]);
    }
    if (want_q) {
      if (lq[r] != 0) atomicAdd(reinterpret_cast<unsigned long long *>(&q_all[i]), (unsigned long long)lq[r]);
      for (int gi = 0; gi < n_groups; ++gi) {
        const long long q = lq[(1 + gi) * nreg + r];
        if (q != 0) atomicAdd(reinterpret_cast<unsigned long long *>(&qg[(int64_t)gi * g.nn + i]), (unsigned long long)q);
      }
    }
  }
}

// v_i = (mv)_i / m_i on active nodes; scene-BC group of each DOF (lowest
// group selecting the node whose mask holds the component).
template <int D>
__global__ void k_p2g_final(GridDev g, const double *gm, double *gv, const long long *qg, SceneBC bc,
                            long long tau_q, int8_t *bcg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nn) return;
  const double m = gm[i];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (m > 0.0) gv[i * D + a] /= m;
    int8_t gsel = -1;
    if (m > 0.0) {
      for (int gi = 0; gi < bc.n_groups; ++gi) {
        if (((bc.mask[gi] >> a) & 1) && qg[(int64_t)gi * g.nn + i] > tau_q) {
          gsel = (int8_t)gi;
          break;
        }
      }
    }
    bcg[i * D + a] = gsel;
  }
}

// ====================================================================== G2P
// APIC G2P with v_i = u_i / dt (Eqs. g2p_v, g2p_B), F <- (I + sum u_i gradN^T) F
// (Eq. F_update) and x <- x + dt v_p (Eq. advection).
template <int D, typename TB>
__global__ void k_g2p(int n, GridDev g, const double *gm, const double *u, double dt, double *x, TB *v, TB *B,
                      TB *F, int64_t cap, int *err) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double xp[D];
#pragma unroll
  for (int a = 0; a < D; ++a) xp[a] = x[a * cap + p];
  Stencil<D> st;
  if (!stencil_eval<D>(xp, g, st)) atomicOr(err, kErrOutOfGrid);
  double vp[D], Bp[D * D], G[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a) vp[a] = 0.0;
#pragma unroll
  for (int k = 0; k < D * D; ++k) {
    Bp[k] = 0.0;
    G[k] = 0.0;
  }
  const double idt = 1.0 / dt;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int i = node_flat<D>(g, idx);
    if (!(gm[i] > 0.0)) continue;
    const double N = stencil_N<D>(st, k);
    double gN[D], dxv[D], ui[D];
    stencil_gradN<D>(st, k, gN);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      dxv[a] = ((double)k[a] - st.f[a]) * g.dx;
      ui[a] = u[i * D + a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double vi = ui[a] * idt;
      vp[a] += N * vi;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        Bp[a * D + b] += N * vi * dxv[b];
        G[a * D + b] += ui[a] * gN[b];
      }
    }
  }
  double Fp[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) Fp[k] = (double)F[k * cap + p];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double t = Fp[a * D + b];
#pragma unroll
      for (int e = 0; e < D; ++e) t += G[a * D + e] * Fp[e * D + b];
      F[(a * D + b) * cap + p] = (TB)t;
      B[(a * D + b) * cap + p] = (TB)Bp[a * D + b];
    }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    v[a * cap + p] = (TB)vp[a];
    x[a * cap + p] = xp[a] + dt * vp[a];
  }
}

// ====================================================================== Dirichlet data
// Prescribed displacement of scene group gi on DOF (i, a) over dt.
template <int D>
__device__ inline double scene_value(const SceneBC &bc, int gi, const GridDev &g, int i, int a, double dt) {
  if (bc.kind[gi] == 0) return 0.0;
  if (bc.kind[gi] == 1) return dt * bc.param[gi][a];
  if constexpr (D == 3) {
    int idx[3];
    double xi[3];
    node_unflat<D>(g, i, idx);
    node_position<D>(g, idx, xi);
    const double *pr = bc.param[gi];
    const double th = pr[6] * dt;
    const double r[3] = {xi[0] - pr[0], xi[1] - pr[1], xi[2] - pr[2]};
    const double kk[3] = {pr[3], pr[4], pr[5]};
    const double kr = kk[0] * r[0] + kk[1] * r[1] + kk[2] * r[2];
    const double kxr[3] = {kk[1] * r[2] - kk[2] * r[1], kk[2] * r[0] - kk[0] * r[2], kk[0] * r[1] - kk[1] * r[0]};
    const double ct = cos(th), sn = sin(th);
    return r[a] * ct + kxr[a] * sn + kk[a] * kr * (1.0 - ct) - r[a];
  }
  return 0.0;
}

// Free-DOF mask and initial iterate: inactive -> 0; scene DOF -> scene value;
// Schwarz receiver -> dt * v_bc; free -> dt * v^n.  Partial sums of the node
// mass for the Newton tolerance floor.
template <int D>
__global__ void k_bc_init(GridDev g, const double *gm, const double *gv, const int8_t *bcg, const uint8_t *recv,
                          const double *vbc, int use_schwarz, SceneBC bc, double dt, uint8_t *fr, double *u,
                          double *part_m) {
  __shared__ double red[kBlock / 64];
  double msum = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.nn; i += gridDim.x * blockDim.x) {
    const double m = gm[i];
    const bool act = m > 0.0;
    if (act) msum += m;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = i * D + a;
      uint8_t f = 0;
      double val = 0.0;
      if (act) {
        const int gi = bcg[k];
        if (gi >= 0) {
          val = scene_value<D>(bc, gi, g, i, a, dt);
        } else if (use_schwarz && recv[i]) {
          val = dt * vbc[k];
        } else {
          f = 1;
          val = dt * gv[k];
        }
      }
      fr[k] = f;
      u[k] = val;
    }
  }
  const double t = block_sum(msum, red);
  if (threadIdx.x == 0) part_m[blockIdx.x] = t;
}

// ====================================================================== gradient + Hessian
// Per particle at the iterate u: F = (I + sum u_i gradN_i^T) F^n and P(F) in
// FP64; the gradient V P F^nT gradN_i is scattered (FP64).  With want_hess
// the particle's tangent A = dP/dF (PSD-projected when asked) is evaluated in
// the bulk type TB, folded with F^n and V, Atil = V C^T A C with C: G -> G F^n,
// stored packed, and its contribution to the Jacobi diagonal is scattered.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_grad_hess(TileGeom tg, GridDev g, const int *cell_start,
                                                      const double *x, const TB *F, const double *vol,
                                                      const int *mat, const double *mu_t, const double *lam_t,
                                                      int64_t cap, const double *u, int want_hess, int project,
                                                      double *gg, TB *gdiag, TB *Atil, int *err) {
  constexpr int n = D * D;
  constexpr int ns = n * (n + 1) / 2;
  extern __shared__ double lds[];
  const int t = tile_of_block(tg, blockIdx.x);
  int p0, p1, org[3];
  if (!tile_range(tg, cell_start, t, p0, p1, org) || p0 == p1) return;
  const int nreg = tg.nreg;
  double *lu = lds;
  double *lg = lds + D * nreg;
  double *ld = lds + 2 * D * nreg;
  for (int r = threadIdx.x; r < nreg; r += kBlock) {
    const int i = region_node<D>(tg, g, org, r);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      lu[a * nreg + r] = (i >= 0) ? u[i * D + a] : 0.0;
      lg[a * nreg + r] = 0.0;
      ld[a * nreg + r] = 0.0;
    }
  }
  __syncthreads();
  for (int p = p0 + threadIdx.x; p < p1; p += kBlock) {
    double xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = x[a * cap + p];
    Stencil<D> st;
    stencil_eval<D>(xp, g, st);
    int l[3];
    if (!local_base<D>(tg, st, org, l)) {
      atomicOr(err, kErrTile);
      continue;
    }
    double Fn[n], Gu[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
      Fn[k] = (double)F[k * cap + p];
      Gu[k] = 0.0;
    }
#pragma unroll
    for (int s = 0; s < stencil_count<D>(); ++s) {
      int k[3];
      stencil_offset<D>(s, k);
      double gN[D];
      stencil_gradN<D>(st, k, gN);
      const int r = region_slot<D>(tg, l, k);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double ua = lu[a * nreg + r];
#pragma unroll
        for (int b = 0; b < D; ++b) Gu[a * D + b] += ua * gN[b];
      }
    }
    double Fc[n];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        double tv = Fn[a * D + b];
#pragma unroll
        for (int e = 0; e < D; ++e) tv += Gu[a * D + e] * Fn[e * D + b];
        Fc[a * D + b] = tv;
      }
    const int mt = mat[p];
    const double mu = mu_t[mt], lam = lam_t[mt], V = vol[p];
    double P[n];
    if (!nh_stress<D, double>(Fc, mu, lam, P, nullptr)) {
      atomicOr(err, kErrInverted);
      continue;
    }
    // T = V P F^nT
    double T[n];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        double tv = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) tv += P[a * D + c] * Fn[b * D + c];
        T[a * D + b] = V * tv;
      }
    TB At[ns];
    if (want_hess) {
      TB Fb[n], Fnb[n], A[n * n];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        Fb[k] = (TB)Fc[k];
        Fnb[k] = (TB)Fn[k];
      }
      nh_stress<D, TB>(Fb, (TB)mu, (TB)lam, nullptr, A);
      if (project) psd_project<n, TB>(A);
      // T1[(ab),(cz)] = sum_y F_by A[(ay),(cz)];  Atil[(ab),(ce)] = V sum_z T1[(ab),(cz)] F_ez
      TB T1[n * n];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b)
#pragma unroll
          for (int q = 0; q < n; ++q) {
            TB tv = TB(0);
#pragma unroll
            for (int y = 0; y < D; ++y) tv += Fnb[b * D + y] * A[(a * D + y) * n + q];
            T1[(a * D + b) * n + q] = tv;
          }
      const TB Vb = (TB)V;
#pragma unroll
      for (int rr = 0; rr < n; ++rr)
#pragma unroll
        for (int c = 0; c < D; ++c)
#pragma unroll
          for (int e = 0; e < D; ++e) {
            const int cc = c * D + e;
            if (cc < rr) continue;
            TB tv = TB(0);
#pragma unroll
            for (int z = 0; z < D; ++z) tv += T1[rr * n + c * D + z] * Fnb[e * D + z];
            At[sym_index<n>(rr, cc)] = Vb * tv;
          }
#pragma unroll
      for (int k = 0; k < ns; ++k) Atil[k * cap + p] = At[k];
    }
#pragma unroll
    for (int s = 0; s < stencil_count<D>(); ++s) {
      int k[3];
      stencil_offset<D>(s, k);
      double gN[D];
      stencil_gradN<D>(st, k, gN);
      const int r = region_slot<D>(tg, l, k);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double tv = 0.0;
#pragma unroll
        for (int b = 0; b < D; ++b) tv += T[a * D + b] * gN[b];
        atomicAdd(&lg[a * nreg + r], tv);
      }
      if (want_hess) {
        TB gb[D];
#pragma unroll
        for (int a = 0; a < D; ++a) gb[a] = (TB)gN[a];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          TB dv = TB(0);
#pragma unroll
          for (int b = 0; b < D; ++b)
#pragma unroll
            for (int e = 0; e < D; ++e) {
              const int r1 = a * D + b, c1 = a * D + e;
              const TB av = (r1 <= c1) ? At[sym_index<n>(r1, c1)] : At[sym_index<n>(c1, r1)];
              dv += av * gb[b] * gb[e];
            }
          atomicAdd(&ld[a * nreg + r], (double)dv);
        }
      }
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < nreg; r += kBlock) {
    const int i = region_node<D>(tg, g, org, r);
    if (i < 0) continue;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double gv = lg[a * nreg + r];
      if (gv != 0.0) atomicAdd(&gg[i * D + a], gv);
      if (want_hess) {
        const double dv = ld[a * nreg + r];
        if (dv != 0.0) atomicAdd(&gdiag[i * D + a], (TB)dv);
      }
    }
  }
}

// Node part of the gradient: + m/dt^2 (u - dt v^n) - m g on active nodes,
// masked to free DOFs; partial |g|^2.  With want_hess the Jacobi diagonal
// becomes scatter + m/dt^2 (1 on non-free DOFs).
template <int D, typename TB>
__global__ void k_grad_node(GridDev g, const double *gm, const double *gv, const double *u, const uint8_t *fr,
                            double dt, double gx, double gy, double gz, double *gg, TB *gdiag, int want_hess,
                            double *part) {
  __shared__ double red[kBlock / 64];
  const double grav[3] = {gx, gy, gz};
  const double idt2 = 1.0 / (dt * dt);
  double s2 = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.nn; i += gridDim.x * blockDim.x) {
    const double m = gm[i];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = i * D + a;
      double gval = gg[k];
      if (m > 0.0) gval += m * idt2 * (u[k] - dt * gv[k]) - m * grav[a];
      if (!fr[k]) gval = 0.0;
      gg[k] = gval;
      s2 += gval * gval;
      if (want_hess) gdiag[k] = fr[k] ? (TB)((double)gdiag[k] + m * idt2) : TB(1);
    }
  }
  const double t = block_sum(s2, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// ====================================================================== CG
// The CG vectors r, z, p, Hp, del and the Jacobi diagonal are stored in the
// bulk type TB (FP32 in the mixed path); scalars, dot products and the
// vector arithmetic are FP64.

// New search direction z + beta p_prev, rounded to the storage type.  Written
// without FMA contraction so the LDS copy and the stored copy agree bit for bit.
template <typename TB>
__device__ inline TB cg_direction(TB z, double beta, TB pp) {
#pragma clang fp contract(off)
  const double t = beta * (double)pp;
  return (TB)((double)z + t);
}

// r = -g, z = r / D on free DOFs; search-direction buffers, direction and
// product cleared; partial (r, z) and (r, r).
template <int D, typename TB>
__global__ void k_cg_init(int ndof, const double *gg, const TB *gdiag, const uint8_t *fr, TB *r, TB *z, TB *p0,
                          TB *p1, TB *del, TB *Hp, double *part_rz, double *part_rr, CgState *S) {
  __shared__ double red[kBlock / 64];
  double rz = 0.0, rr = 0.0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ndof; k += gridDim.x * blockDim.x) {
    const bool f = fr[k];
    const TB rv = f ? (TB)(-gg[k]) : TB(0);
    const TB zv = f ? (TB)((double)rv / (double)gdiag[k]) : TB(0);
    r[k] = rv;
    z[k] = zv;
    p0[k] = TB(0);
    p1[k] = TB(0);
    del[k] = TB(0);
    Hp[k] = TB(0);
    if (f) {
      rz += (double)rv * (double)zv;
      rr += (double)rv * (double)rv;
    }
  }
  const double a = block_sum(rz, red);
  const double b = block_sum(rr, red);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = a;
    part_rr[blockIdx.x] = b;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->iter = 0;
    S->done = 0;
    S->knext = 0;
    S->kcur = 0;
  }
}

// Sum over a workgroup of two values at once (every thread gets both).
__device__ inline void block_sum2(double &a, double &b, double *lds8) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    lds8[w] = a;
    lds8[4 + w] = b;
  }
  __syncthreads();
  a = lds8[0] + lds8[1] + lds8[2] + lds8[3];
  b = lds8[4] + lds8[5] + lds8[6] + lds8[7];
}

// CG iteration, first half.  The iteration index k comes from the device
// state (so a chunk of iterations can be replayed with fixed arguments).
// Every workgroup sums the (r, z) and (r, r) partials of the previous update
// in the same order, tests |r| <= rtol |r0| (and k < max_cg), and forms beta.
// The search direction p = z + beta p_prev is formed on the fly (tile regions
// in LDS, owned DOFs stored to p_cur).  The particle part scatters
// Hp = sum_p Atil:G gradN and accumulates the curvature
// p^T H p = sum_p G:Atil:G + sum_i m_i/dt^2 |p_i|^2, so the product and its
// curvature complete in one pass.  All global loads that do not depend on
// beta are issued before the reduction so their latencies overlap.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_cg_hvp(TileGeom tg, GridDev g, const int *cell_start, const double *x,
                                                   const TB *Atil, int64_t cap, const double *gm, double dt,
                                                   int ndof, const TB *z, TB *pA, TB *pB, TB *Hp,
                                                   const double *part_rz, const double *part_rr, int n_part,
                                                   double rtol, int max_cg, double *part_q, CgState *S) {
  constexpr int n = D * D;
  constexpr int ns = n * (n + 1) / 2;
  extern __shared__ double lds[];
  __shared__ double red[8];
  const int tid = threadIdx.x;
  const int it = S->knext;
  const TB *pprev = (it & 1) ? pA : pB;
  TB *pcur = (it & 1) ? pB : pA;
  // tile and its particle range
  const int t = tile_of_block(tg, blockIdx.x);
  int p0 = 0, p1 = 0, org[3] = {0, 0, 0};
  const bool tile_ok = tile_range(tg, cell_start, t, p0, p1, org) && p0 < p1;
  const int nreg = tg.nreg;
  // --- independent loads
  double prz = 0.0, prr = 0.0;
  for (int i = tid; i < n_part; i += kBlock) {
    prz += part_rz[i];
    prr += part_rr[i];
  }
  const int k0 = blockIdx.x * kBlock + tid;
  TB nz = TB(0), npv = TB(0);
  double nm = 0.0;
  if (k0 < ndof) {
    nz = z[k0];
    npv = pprev[k0];
    nm = gm[k0 / D];
  }
  int ri = -1;
  TB rzv[D], rpv[D];
  if (tile_ok && tid < nreg) {
    ri = region_node<D>(tg, g, org, tid);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      rzv[a] = (ri >= 0) ? z[ri * D + a] : TB(0);
      rpv[a] = (ri >= 0) ? pprev[ri * D + a] : TB(0);
    }
  }
  const int pp = p0 + tid;
  const bool have_p = tile_ok && pp < p1;
  double xp[D];
  TB At[ns];
  if (have_p) {
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = x[a * cap + pp];
#pragma unroll
    for (int k = 0; k < ns; ++k) At[k] = Atil[k * cap + pp];
  }
  // --- reduction, convergence test, beta
  block_sum2(prz, prr, red);
  const double rz_new = prz, rr = prr;
  const double rr0 = (it == 0) ? rr : S->rr0;
  const bool done = (it >= max_cg) || ((it == 0) ? !(rr0 > 0.0) : (sqrt(rr) <= rtol * sqrt(rr0)));
  if (blockIdx.x == 0 && tid == 0) {
    if (it == 0) S->rr0 = rr0;
    if (done) S->done = 1;
    S->rz[it & 1] = rz_new;
    S->kcur = it;
  }
  if (done || S->done) return;
  const double beta = (it == 0) ? 0.0 : rz_new / S->rz[(it + 1) & 1];
  const double mdt = 1.0 / (dt * dt);
  double q = 0.0;
  // node part: owned DOFs of the new direction and its mass term
  if (k0 < ndof) {
    const TB pv = cg_direction<TB>(nz, beta, npv);
    pcur[k0] = pv;
    q += nm * mdt * (double)pv * (double)pv;
  }
  for (int k = k0 + gridDim.x * kBlock; k < ndof; k += gridDim.x * kBlock) {
    const TB pv = cg_direction<TB>(z[k], beta, pprev[k]);
    pcur[k] = pv;
    q += gm[k / D] * mdt * (double)pv * (double)pv;
  }
  if (tile_ok) {
    double *lh = lds;
    TB *lp = reinterpret_cast<TB *>(lds + D * nreg);
    if (tid < nreg) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lp[a * nreg + tid] = (ri >= 0) ? cg_direction<TB>(rzv[a], beta, rpv[a]) : TB(0);
        lh[a * nreg + tid] = 0.0;
      }
    }
    for (int r = tid + kBlock; r < nreg; r += kBlock) {
      const int i = region_node<D>(tg, g, org, r);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lp[a * nreg + r] = (i >= 0) ? cg_direction<TB>(z[i * D + a], beta, pprev[i * D + a]) : TB(0);
        lh[a * nreg + r] = 0.0;
      }
    }
    __syncthreads();
    for (int p = pp; p < p1; p += kBlock) {
      if (p != pp) {
#pragma unroll
        for (int a = 0; a < D; ++a) xp[a] = x[a * cap + p];
#pragma unroll
        for (int k = 0; k < ns; ++k) At[k] = Atil[k * cap + p];
      }
      Stencil<D> st;
      stencil_eval<D>(xp, g, st);
      int l[3];
      if (!local_base<D>(tg, st, org, l)) continue;
      TB G[n];
#pragma unroll
      for (int k = 0; k < n; ++k) G[k] = TB(0);
#pragma unroll
      for (int s = 0; s < stencil_count<D>(); ++s) {
        int k[3];
        stencil_offset<D>(s, k);
        double gN[D];
        stencil_gradN<D>(st, k, gN);
        const int r = region_slot<D>(tg, l, k);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const TB pa = lp[a * nreg + r];
#pragma unroll
          for (int b = 0; b < D; ++b) G[a * D + b] += pa * (TB)gN[b];
        }
      }
      TB T[n];
      TB qp = TB(0);
#pragma unroll
      for (int rr2 = 0; rr2 < n; ++rr2) {
        TB tv = TB(0);
#pragma unroll
        for (int cc = 0; cc < n; ++cc)
          tv += ((rr2 <= cc) ? At[sym_index<n>(rr2, cc)] : At[sym_index<n>(cc, rr2)]) * G[cc];
        T[rr2] = tv;
        qp += G[rr2] * tv;
      }
      q += (double)qp;
#pragma unroll
      for (int s = 0; s < stencil_count<D>(); ++s) {
        int k[3];
        stencil_offset<D>(s, k);
        double gN[D];
        stencil_gradN<D>(st, k, gN);
        const int r = region_slot<D>(tg, l, k);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          TB tv = TB(0);
#pragma unroll
          for (int b = 0; b < D; ++b) tv += T[a * D + b] * (TB)gN[b];
          atomicAdd(&lh[a * nreg + r], (double)tv);
        }
      }
    }
    __syncthreads();
    for (int r = tid; r < nreg; r += kBlock) {
      const int i = (r == tid) ? ri : region_node<D>(tg, g, org, r);
      if (i < 0) continue;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double hv = lh[a * nreg + r];
        if (hv != 0.0) atomicAdd(&Hp[i * D + a], (TB)hv);
      }
    }
  }
  const double tq = block_sum(q, red);
  if (tid == 0) part_q[blockIdx.x] = tq;
}

// CG iteration, second half: alpha = (r, z) / p^T H p; del += alpha p,
// r -= alpha H p (H p = scatter + m/dt^2 p), z = r / D on free DOFs; the
// scatter buffer is cleared for the next product; partial (r, z), (r, r).
// Node data are loaded before the curvature partials are reduced.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_cg_update(int ndof, const double *gm, double dt, const uint8_t *fr,
                                                      const TB *gdiag, const TB *pA, const TB *pB, TB *Hp, TB *r,
                                                      TB *z, TB *del, const double *part_q, int n_q,
                                                      double *part_rz, double *part_rr, CgState *S) {
  __shared__ double red[8];
  const int tid = threadIdx.x;
  if (S->done) return;
  const int it = S->kcur;
  const TB *pcur = (it & 1) ? pB : pA;
  double pq = 0.0;
  for (int i = tid; i < n_q; i += kBlock) pq += part_q[i];
  const int k0 = blockIdx.x * kBlock + tid;
  double hs = 0.0, pv = 0.0, rv = 0.0, dv = 0.0, dg = 1.0, m = 0.0;
  bool f = false;
  if (k0 < ndof) {
    f = fr[k0];
    hs = (double)Hp[k0];
    pv = (double)pcur[k0];
    rv = (double)r[k0];
    dv = (double)del[k0];
    dg = (double)gdiag[k0];
    m = gm[k0 / D];
  }
  pq = block_sum(pq, red);
  if (!(pq > 0.0)) {
    if (blockIdx.x == 0 && tid == 0) S->done = 1;
    return;
  }
  const double alpha = S->rz[it & 1] / pq;
  const double mdt = 1.0 / (dt * dt);
  double rz = 0.0, rr = 0.0;
  if (k0 < ndof) {
    Hp[k0] = TB(0);
    if (f) {
      const double hv = hs + m * mdt * pv;
      del[k0] = (TB)(dv + alpha * pv);
      const TB rn = (TB)(rv - alpha * hv);
      r[k0] = rn;
      const TB zv = (TB)((double)rn / dg);
      z[k0] = zv;
      rz += (double)rn * (double)zv;
      rr += (double)rn * (double)rn;
    }
  }
  for (int k = k0 + gridDim.x * kBlock; k < ndof; k += gridDim.x * kBlock) {
    const double h2 = (double)Hp[k];
    Hp[k] = TB(0);
    if (!fr[k]) continue;
    const double p2 = (double)pcur[k];
    const double hv = h2 + gm[k / D] * mdt * p2;
    del[k] = (TB)((double)del[k] + alpha * p2);
    const TB rn = (TB)((double)r[k] - alpha * hv);
    r[k] = rn;
    const TB zv = (TB)((double)rn / (double)gdiag[k]);
    z[k] = zv;
    rz += (double)rn * (double)zv;
    rr += (double)rn * (double)rn;
  }
  block_sum2(rz, rr, red);
  if (tid == 0) {
    part_rz[blockIdx.x] = rz;
    part_rr[blockIdx.x] = rr;
  }
  if (blockIdx.x == 0 && tid == 0) {
    S->iter = it + 1;
    S->knext = it + 1;
  }
}

// ====================================================================== line search
// Per-particle part of E(u + alpha del) - E(u) in cancellation-free form:
// V [mu/2 (2 F:Dm + Dm:Dm) - mu L + lam/2 L (2 ln J + L)], L = log1p(dJ / J),
// dJ = det(F + Dm) - det F expanded in powers of Dm; +inf on inversion.
template <int D, typename TB>
__global__ void k_delta_energy_p(int np, GridDev g, const double *x, const TB *F, const double *vol,
                                 const int *mat, const double *mu_t, const double *lam_t, int64_t cap,
                                 const double *u, const TB *del, double alpha, double *part) {
  constexpr int n = D * D;
  __shared__ double red[kBlock / 64];
  double e = 0.0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
    double xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = x[a * cap + p];
    Stencil<D> st;
    stencil_eval<D>(xp, g, st);
    double Gu[n], Gd[n], Fn[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
      Gu[k] = 0.0;
      Gd[k] = 0.0;
      Fn[k] = (double)F[k * cap + p];
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
        const double ua = u[i * D + a], da = (double)del[i * D + a];
#pragma unroll
        for (int b = 0; b < D; ++b) {
          Gu[a * D + b] += ua * gN[b];
          Gd[a * D + b] += da * gN[b];
        }
      }
    }
    double Fc[n], Dm[n];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        double tf = Fn[a * D + b], td = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          tf += Gu[a * D + c] * Fn[c * D + b];
          td += Gd[a * D + c] * Fn[c * D + b];
        }
        Fc[a * D + b] = tf;
        Dm[a * D + b] = alpha * td;
      }
    const double J = det<D, double>(Fc);
    double CF[n];
    cofactor<D, double>(Fc, CF);
    double dJ = 0.0;
#pragma unroll
    for (int k = 0; k < n; ++k) dJ += CF[k] * Dm[k];
    if constexpr (D == 3) {
      double CD[n];
      cofactor<D, double>(Dm, CD);
#pragma unroll
      for (int k = 0; k < n; ++k) dJ += Fc[k] * CD[k];
    }
    dJ += det<D, double>(Dm);
    if (!(J > 0.0) || !(J + dJ > 0.0)) {
      e = HUGE_VAL;
      continue;
    }
    const double lnJ = log(J);
    const double L = log1p(dJ / J);
    double FD = 0.0, DD = 0.0;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      FD += Fc[k] * Dm[k];
      DD += Dm[k] * Dm[k];
    }
    const int mt = mat[p];
    const double mu = mu_t[mt], lam = lam_t[mt];
    e += vol[p] * (0.5 * mu * (2.0 * FD + DD) - mu * L + 0.5 * lam * L * (2.0 * lnJ + L));
  }
  const double t = block_sum(e, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Node part: m/(2 dt^2) (2 alpha (u - dt v^n).del + alpha^2 |del|^2) - alpha m g.del.
template <int D, typename TB>
__global__ void k_delta_energy_n(GridDev g, const double *gm, const double *gv, const double *u, const TB *del,
                                 double dt, double alpha, double gx, double gy, double gz, double *part) {
  __shared__ double red[kBlock / 64];
  const double grav[3] = {gx, gy, gz};
  double e = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.nn; i += gridDim.x * blockDim.x) {
    const double m = gm[i];
    if (!(m > 0.0)) continue;
    double rd = 0.0, dd = 0.0, gd = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double dv = (double)del[i * D + a];
      rd += (u[i * D + a] - dt * gv[i * D + a]) * dv;
      dd += dv * dv;
      gd += grav[a] * dv;
    }
    e += m / (2.0 * dt * dt) * (2.0 * alpha * rd + alpha * alpha * dd) - alpha * m * gd;
  }
  const double t = block_sum(e, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename TB>
__global__ void k_axpy(int n, double alpha, const TB *xv, double *y) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    y[k] += alpha * (double)xv[k];
}
template __global__ void k_axpy<double>(int, double, const double *, double *);
template __global__ void k_axpy<float>(int, double, const float *, double *);

// ====================================================================== interface
// Fixed-point node mass of the boundary-layer particles (Eq. boundary_grid_set).
template <int D>
__global__ void k_qbnd(int np, GridDev g, const double *x, const double *mass, const uint8_t *flags, int64_t cap,
                       double scale, long long *q_bnd) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np || !(flags[p] & 1u)) return;
  double xp[D];
#pragma unroll
  for (int a = 0; a < D; ++a) xp[a] = x[a * cap + p];
  Stencil<D> st;
  stencil_eval<D>(xp, g, st);
  const double mq = mass[p] * scale;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const long long q = fixed_mass(stencil_N<D>(st, k), mq);
    if (q != 0) atomicAdd(reinterpret_cast<unsigned long long *>(&q_bnd[node_flat<D>(g, idx)]), (unsigned long long)q);
  }
}

__global__ void k_gamma(int nn, const long long *q_bnd, const double *gm, long long tau_q, uint8_t *gamma,
                        uint8_t *recv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const uint8_t gsel = (q_bnd[i] > tau_q && gm[i] > 0.0) ? 1 : 0;
  gamma[i] = gsel;
  recv[i] = gsel;
}

// Overlap arbitration (Eq. overlap_donor): a coarse boundary node whose
// lattice point is a fine boundary node is ambiguous; the larger fixed-point
// node mass donates (ties: the coarse side) and leaves its receiver set.
template <int D>
__global__ void k_arbitrate(GridDev gB, GridDev gS, const uint8_t *gammaB, const uint8_t *gammaS,
                            const long long *qB, const long long *qS, uint8_t *recvB, uint8_t *recvS, int *n_amb) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= gB.nn || !gammaB[I]) return;
  int iB[3], jS[3];
  node_unflat<D>(gB, I, iB);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const long long L = gB.origin_q[a] + (long long)iB[a] * gB.dx_q;
    const long long t = L - gS.origin_q[a];
    if (t < 0 || t % gS.dx_q != 0 || t / gS.dx_q >= gS.n[a]) return;
    jS[a] = (int)(t / gS.dx_q);
  }
  const int j = node_flat<D>(gS, jS);
  if (!gammaS[j]) return;
  atomicAdd(n_amb, 1);
  if (qB[I] >= qS[j])
    recvB[I] = 0;
  else
    recvS[j] = 0;
}

// Pi_{S->B} numerator and denominator: every active fine node j scatters
// m_j N_I(x_j) and m_j v_j N_I(x_j) onto its coarse stencil.
template <int D>
__global__ void k_project_scatter(GridDev gS, GridDev gB, const double *mS, const double *vS, double *num,
                                  double *den, int *err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= gS.nn) return;
  const double m = mS[j];
  if (!(m > 0.0)) return;
  int jS[3];
  double xj[D];
  node_unflat<D>(gS, j, jS);
  node_position<D>(gS, jS, xj);
  Stencil<D> st;
  if (!stencil_eval<D>(xj, gB, st)) {
    atomicOr(err, kErrOutOfGrid);
    return;
  }
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int I = node_flat<D>(gB, idx);
    const double w = m * stencil_N<D>(st, k);
    atomicAdd(&den[I], w);
#pragma unroll
    for (int a = 0; a < D; ++a) atomicAdd(&num[I * D + a], w * vS[j * D + a]);
  }
}

template <int D>
__global__ void k_project_final(int nn, const uint8_t *recv, const double *num, const double *den, double eps_tol,
                                double *out) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nn) return;
  const bool rc = recv[I];
#pragma unroll
  for (int a = 0; a < D; ++a) out[I * D + a] = rc ? num[I * D + a] / (den[I] + eps_tol) : 0.0;
}

// I_{B->S} at the fine receivers (Eq. interp_BtoS).
template <int D>
__global__ void k_interp(GridDev gB, GridDev gS, const double *mB, const double *vB, const uint8_t *recvS,
                         double *out, int *err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= gS.nn) return;
  double acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = 0.0;
  if (recvS[j]) {
    int jS[3];
    double xj[D];
    node_unflat<D>(gS, j, jS);
    node_position<D>(gS, jS, xj);
    Stencil<D> st;
    if (!stencil_eval<D>(xj, gB, st)) {
      atomicOr(err, kErrOutOfGrid);
    } else {
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
        for (int a = 0; a < D; ++a) acc[a] += N * vB[I * D + a];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) out[j * D + a] = acc[a];
}

// T_m (Eq. temporal_interp).
__global__ void k_temporal(int64_t n, double am, const double *vn, const double *vn1, double *out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = (1.0 - am) * vn[k] + am * vn1[k];
}

// v = u / dt on active nodes, 0 elsewhere.
template <int D>
__global__ void k_vel_from_u(int nn, const double *gm, const double *u, double dt, double *v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const bool act = gm[i] > 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) v[i * D + a] = act ? u[i * D + a] / dt : 0.0;
}

// Partial sums over receiver nodes of |a - b|^2 and |a|^2 (Eq.
// convergence_residuals).
template <int D>
__global__ void k_resid(int nn, const uint8_t *recv, const double *a, const double *b, double *part) {
  __shared__ double red[kBlock / 64];
  double s = 0.0, t = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += gridDim.x * blockDim.x) {
    if (!recv[i]) continue;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double e = a[i * D + c] - b[i * D + c];
      s += e * e;
      t += a[i * D + c] * a[i * D + c];
    }
  }
  const double x1 = block_sum(s, red);
  const double x2 = block_sum(t, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = x1;
    part[2 * blockIdx.x + 1] = x2;
  }
}

// ====================================================================== instantiations
#define OSMPM_INST_D(D)                                                                                            \
  template __global__ void k_keys<D>(int, const double *, int64_t, GridDev, TileGeom, int *, int *, int *);        \
  template __global__ void k_p2g_final<D>(GridDev, const double *, double *, const long long *, SceneBC,          \
                                          long long, int8_t *);                                                    \
  template __global__ void k_bc_init<D>(GridDev, const double *, const double *, const int8_t *, const uint8_t *, \
                                        const double *, int, SceneBC, double, uint8_t *, double *, double *);     \
  template __global__ void k_qbnd<D>(int, GridDev, const double *, const double *, const uint8_t *, int64_t,       \
                                     double, long long *);                                                         \
  template __global__ void k_arbitrate<D>(GridDev, GridDev, const uint8_t *, const uint8_t *, const long long *,   \
                                          const long long *, uint8_t *, uint8_t *, int *);                        \
  template __global__ void k_project_scatter<D>(GridDev, GridDev, const double *, const double *, double *,       \
                                                double *, int *);                                                  \
  template __global__ void k_project_final<D>(int, const uint8_t *, const double *, const double *, double,       \
                                              double *);                                                           \
  template __global__ void k_interp<D>(GridDev, GridDev, const double *, const double *, const uint8_t *,         \
                                       double *, int *);                                                           \
  template __global__ void k_vel_from_u<D>(int, const double *, const double *, double, double *);                 \
  template __global__ void k_resid<D>(int, const uint8_t *, const double *, const double *, double *);

#define OSMPM_INST_DT(D, TB)                                                                                       \
  template __global__ void k_p2g<D, TB>(TileGeom, GridDev, const int *, const double *, const TB *, const TB *,    \
                                        const double *, const uint8_t *, int64_t, int, double, double, int,       \
                                        double *, double *, long long *, long long *, int *);                     \
  template __global__ void k_g2p<D, TB>(int, GridDev, const double *, const double *, double, double *, TB *,      \
                                        TB *, TB *, int64_t, int *);                                               \
  template __global__ void k_grad_hess<D, TB>(TileGeom, GridDev, const int *, const double *, const TB *,          \
                                              const double *, const int *, const double *, const double *,        \
                                              int64_t, const double *, int, int, double *, TB *, TB *, int *);    \
  template __global__ void k_grad_node<D, TB>(GridDev, const double *, const double *, const double *,            \
                                              const uint8_t *, double, double, double, double, double *, TB *,    \
                                              int, double *);                                                      \
  template __global__ void k_cg_init<D, TB>(int, const double *, const TB *, const uint8_t *, TB *, TB *, TB *,    \
                                            TB *, TB *, TB *, double *, double *, CgState *);                     \
  template __global__ void k_cg_hvp<D, TB>(TileGeom, GridDev, const int *, const double *, const TB *, int64_t,    \
                                           const double *, double, int, const TB *, TB *, TB *, TB *,             \
                                           const double *, const double *, int, double, int, double *, CgState *); \
  template __global__ void k_cg_update<D, TB>(int, const double *, double, const uint8_t *, const TB *,           \
                                              const TB *, const TB *, TB *, TB *, TB *, TB *, const double *,     \
                                              int, double *, double *, CgState *);                                \
  template __global__ void k_delta_energy_p<D, TB>(int, GridDev, const double *, const TB *, const double *,       \
                                                   const int *, const double *, const double *, int64_t,          \
                                                   const double *, const TB *, double, double *);                 \
  template __global__ void k_delta_energy_n<D, TB>(GridDev, const double *, const double *, const double *,       \
                                                   const TB *, double, double, double, double, double, double *);

OSMPM_INST_D(2)
OSMPM_INST_D(3)
OSMPM_INST_DT(2, double)
OSMPM_INST_DT(2, float)
OSMPM_INST_DT(3, double)
OSMPM_INST_DT(3, float)

}  // namespace osmpm
