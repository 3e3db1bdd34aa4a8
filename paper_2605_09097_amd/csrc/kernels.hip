// OS-MPM kernels for gfx950 (wave64, 256-thread workgroups), batched over
// domains: blockIdx.y selects the domain, blockIdx.x the block inside it.
//
// Particle-to-grid style kernels (P2G, gradient/tangent build, CG
// Hessian-vector product) run one workgroup per tile of cells: the particles
// of a tile are contiguous after the binning sort, their 3^d stencils touch
// the (T+2)^d nodes of the tile region, which is staged in LDS (gathers) and
// accumulated in FP64 LDS with LDS atomics (scatters) before one pass of
// global atomics per node.  Node kernels are grid-stride loops over DOFs.
// Reductions go through per-workgroup partials that the consumer sums in a
// fixed order, so every scalar is deterministic run to run.  Decision
// kernels advance each domain's Newton / line-search state on the device.
#include "kernels.hpp"

namespace osmpm {

// ====================================================================== misc
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(int64_t n, T v, T *a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
template __global__ void k_fill<double>(int64_t, double, double *);
template __global__ void k_fill<float>(int64_t, float, float *);
template __global__ void k_fill<int>(int64_t, int, int *);
template __global__ void k_fill<long long>(int64_t, long long, long long *);
template __global__ void k_fill<uint8_t>(int64_t, uint8_t, uint8_t *);

// [n][c] (caller layout, FP64) -> [c][cap] (library layout, storage type T).
// With eye = D + 1 the rows are a D x D matrix and the identity is taken
// off the diagonal rows (r % eye == 0) in FP64 before rounding: F in, H out.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_aos_to_soa(int64_t n, int c, const double *src, T *dst, int64_t cap, int eye) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * c; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / c, r = i % c;
    const double s = (eye && r % eye == 0) ? src[i] - 1.0 : src[i];
    dst[r * cap + p] = (T)s;
  }
}
// Inverse of k_aos_to_soa; eye = D + 1 adds the identity back (H in, F out).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_soa_to_aos(int64_t n, int c, const T *src, int64_t cap, double *dst, int eye) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * c; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / c, r = i % c;
    const double s = (double)src[r * cap + p];
    dst[i] = (eye && r % eye == 0) ? s + 1.0 : s;
  }
}
template __global__ void k_aos_to_soa<double>(int64_t, int, const double *, double *, int64_t, int);
template __global__ void k_aos_to_soa<float>(int64_t, int, const double *, float *, int64_t, int);
template __global__ void k_soa_to_aos<double>(int64_t, int, const double *, int64_t, double *, int);
template __global__ void k_soa_to_aos<float>(int64_t, int, const float *, int64_t, double *, int);

__global__ void __launch_bounds__(kBlock) k_iota(int n, int *a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = i;
}

// flags[i] = bit i of m.
__global__ void __launch_bounds__(kBlock) k_set_flags(int *flags, int n, FlagMask m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = (int)((m.w[i >> 6] >> (i & 63)) & 1u);
}

// T_m (Eq. temporal_interp) on plain arrays.
__global__ void __launch_bounds__(kBlock) k_temporal_1(int64_t n, double am, const double *vn, const double *vn1, double *out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    out[k] = (1.0 - am) * vn[k] + am * vn1[k];
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

// Blocks of a grid-stride particle reduction (also its number of partials).
__device__ inline int particle_blocks(int np) {
  int b = (np + kBlock - 1) / kBlock;
  return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

// ====================================================================== binning
// Zeroes the bin histogram and the P2G targets of every active domain (with
// want_q also the fixed-point masses of the boundary-set selection).
__global__ void __launch_bounds__(kBlock) k_zero_grid(const DomDesc *dd, int want_q) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int nn = dm.g.nn;
  const int stride = gridDim.x * blockDim.x;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  for (int i = i0; i < dm.nk; i += stride) dm.count[i] = 0;
  for (int i = i0; i < nn; i += stride) {
    dm.m[i] = 0.0;
    if (want_q) {
      dm.q_all[i] = 0;
      dm.q_bnd[i] = 0;
      for (int gi = 0; gi < dm.bc.n_groups; ++gi) dm.qg[(int64_t)gi * nn + i] = 0;
    }
  }
  for (int k = i0; k < dm.ndof; k += stride) dm.vn[k] = 0.0;
}

// Tile-major bin key of the particle's base node, and the bin histogram.
template <int D>
__global__ void __launch_bounds__(kBlock) k_keys(const DomDesc *dd, int *err) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= dm.np) return;
  const double *x = dm.pb[*dm.cur].x;
  double xp[D];
#pragma unroll
  for (int a = 0; a < D; ++a) xp[a] = x[a * dm.cap + p];
  Stencil<D> st;
  if (!stencil_eval<D>(xp, dm.g, st)) atomicOr(err, kErrOutOfGrid);
  int t[3] = {0, 0, 0}, l[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    t[a] = st.base[a] / dm.tg.T[a];
    l[a] = st.base[a] % dm.tg.T[a];
  }
  const int tf = t[0] + dm.tg.nt[0] * (t[1] + dm.tg.nt[1] * t[2]);
  const int lf = l[0] + dm.tg.T[0] * (l[1] + dm.tg.T[1] * l[2]);
  const int k = tf * dm.tg.tvol + lf;
  dm.key[p] = k;
  atomicAdd(&dm.count[k], 1);
}

// Bin offsets in three steps, using that bins are tile-major (tvol bins per
// tile): the total of every tile, an exclusive scan of the tile totals, and
// the scan of each tile's bins on top of its tile offset.

// Sum of v over the workgroup (kBlock threads); every thread gets it.
__device__ inline int block_sum_int(int v, int *lds4) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = v;
  __syncthreads();
  return lds4[0] + lds4[1] + lds4[2] + lds4[3];
}

// In-place exclusive scan of a[0, n) by one workgroup of 1024 threads, 4096
// entries per pass (four consecutive ones per thread, so loads and stores
// are coalesced); returns the total to every thread.
__device__ inline int wg_exclusive_scan(int *a, int n) {
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += 4096) {
    int v[4];
    int s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int idx = base + 4 * tid + j;
      v[j] = (idx < n) ? a[idx] : 0;
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
      if (idx < n) a[idx] = excl;
      excl += v[j];
    }
    carry += wsum[15];
    __syncthreads();
  }
  return carry;
}

// ====================================================================== work lists
// Live-tile list of a domain from its bin offsets (after a binning, or after
// a stored binning is restored): the tiles holding particles, in tile order,
// with their particle ranges, dealt to the workgroup slots of a tile launch
// so that each of the 8 XCDs (to which workgroups are dispatched round-robin)
// takes a contiguous band of tiles: slot b takes list entry
// (b mod 8) * per + b / 8, per = ceil(live / 8); the other slots get
// {-1, 0, 0, 0}.  The body, for one workgroup of 1024 threads per domain;
// range(t, p0, p1) gives tile t's particle range.
template <typename Range>
__device__ inline void tile_slots(const DomDesc &dm, Range range) {
  __shared__ int wsum[16];
  const int nt = dm.tg.ntiles, nb = dm.tg.nblocks;
  TileSlot *tl = dm.tl;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int c = 0;
  for (int t = tid; t < nt; t += 1024) {
    int p0, p1;
    range(t, p0, p1);
    c += (p1 > p0) ? 1 : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if (lane == 0) wsum[w] = c;
  __syncthreads();
  int live = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) live += wsum[k];
  __syncthreads();
  const int per = (live + 7) >> 3;
  for (int b = tid; b < nb; b += 1024) {
    const int j = (b & 7) * per + (b >> 3);
    if (!((b >> 3) < per && j < live)) tl[b] = TileSlot{-1, 0, 0, 0};
  }
  int carry = 0;
  for (int base = 0; base < nt; base += 1024) {
    const int t = base + tid;
    int p0 = 0, p1 = 0;
    if (t < nt) range(t, p0, p1);
    const bool f = p1 > p0;
    const unsigned long long bal = __ballot(f);
    if (lane == 0) wsum[w] = (int)__popcll(bal);
    __syncthreads();
    int woff = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int v = wsum[k];
      woff += (k < w) ? v : 0;
      tot += v;
    }
    if (f) {
      const int j = carry + woff + (int)__popcll(bal & ((1ull << lane) - 1ull));
      tl[(j % per) * 8 + j / per] = TileSlot{t, p0, p1, 0};
    }
    carry += tot;
    __syncthreads();
  }
  if (tid == 0) {
    dm.lcnt[0] = live;
    dm.ss->n_tiles_live = live;
  }
}

// The list from the bin offsets of a restored binning.
__global__ void __launch_bounds__(1024) k_tile_list(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int *cs = dm.cell_start;
  const int tvol = dm.tg.tvol;
  tile_slots(dm, [&](int t, int &p0, int &p1) {
    p0 = cs[(int64_t)t * tvol];
    p1 = cs[(int64_t)(t + 1) * tvol];
  });
}

// Active nodes (m > 0) per block of 256 nodes.
__global__ void __launch_bounds__(kBlock) k_node_count(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int nn = dm.g.nn;
  if ((int)blockIdx.x >= (nn + kBlock - 1) / kBlock) return;
  __shared__ int wc[kBlock / 64];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool f = i < nn && dm.m[i] > 0.0;
  const unsigned long long bal = __ballot(f);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (int)__popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) dm.ncnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// Exclusive scan of the per-block active-node counts of a grid of more than
// kNodeListDirect node blocks, in place; one workgroup of 1024 threads per
// domain.  Smaller grids keep their counts (k_node_list sums them itself).
__global__ void __launch_bounds__(1024) k_node_scan(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int nbn = (dm.g.nn + kBlock - 1) / kBlock;
  if (nbn <= kNodeListDirect) return;
  (void)wg_exclusive_scan(dm.ncnt, nbn);
}

// Active-node list in node order: each block of 256 nodes writes its active
// nodes at the number of active nodes in the blocks before it; the last
// block stores the total.  Up to kNodeListDirect blocks that offset is the
// sum of the earlier blocks' counts, formed here (at most 16 loads a thread);
// larger grids read it from k_node_scan, which keeps the work linear in the
// grid size.
__global__ void __launch_bounds__(kBlock) k_node_list(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int nn = dm.g.nn;
  const int nbn = (nn + kBlock - 1) / kBlock;
  if ((int)blockIdx.x >= nbn) return;
  __shared__ int red[kBlock / 64];
  __shared__ int wc[kBlock / 64];
  int off;
  if (nbn > kNodeListDirect) {
    off = dm.ncnt[blockIdx.x];
  } else {
    int sp = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += kBlock) sp += dm.ncnt[j];
    off = block_sum_int(sp, red);
  }
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool f = i < nn && dm.m[i] > 0.0;
  const unsigned long long bal = __ballot(f);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wc[w] = (int)__popcll(bal);
  __syncthreads();
  int woff = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) woff += (k < w) ? wc[k] : 0;
  if (f) dm.nlist[off + woff + (int)__popcll(bal & ((1ull << lane) - 1ull))] = i;
  if ((int)blockIdx.x == nbn - 1 && threadIdx.x == 0) {
    const int total = off + wc[0] + wc[1] + wc[2] + wc[3];
    dm.lcnt[1] = total;
    dm.ss->n_active = total;
  }
}

__global__ void __launch_bounds__(kBlock) k_tile_sum(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active || (int)blockIdx.x >= dm.tg.ntiles) return;
  __shared__ int red[kBlock / 64];
  const int tvol = dm.tg.tvol;
  const int *cnt = dm.count + (size_t)blockIdx.x * tvol;
  int v = 0;
  for (int c = threadIdx.x; c < tvol; c += kBlock) v += cnt[c];
  v = block_sum_int(v, red);
  if (threadIdx.x == 0) dm.tcount[blockIdx.x] = v;
}

// In-place exclusive scan of the tile totals by one workgroup of 1024
// threads; the grand total goes to tcount[ntiles] and to cell_start[nk].
__global__ void __launch_bounds__(1024) k_tile_scan(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int nt = dm.tg.ntiles;
  int *tc = dm.tcount;
  const int carry = wg_exclusive_scan(tc, nt);
  if (threadIdx.x == 0) {
    tc[nt] = carry;
    dm.cell_start[dm.nk] = carry;
  }
  __syncthreads();
  // the live-tile list from the tile offsets just formed
  tile_slots(dm, [&](int t, int &p0, int &p1) {
    p0 = tc[t];
    p1 = tc[t + 1];
  });
}

// Exclusive scan of one tile's bins, offset by the tile's
// start; cursor receives a copy of the offsets for the scatter.
__global__ void __launch_bounds__(kBlock) k_cell_scan(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active || (int)blockIdx.x >= dm.tg.ntiles) return;
  __shared__ int wsum[kBlock / 64];
  const int tvol = dm.tg.tvol;
  const size_t b0 = (size_t)blockIdx.x * tvol;
  const int *cnt = dm.count + b0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int carry = dm.tcount[blockIdx.x];
  for (int base = 0; base < tvol; base += kBlock) {
    const int c = base + tid;
    const int v = (c < tvol) ? cnt[c] : 0;
    int xs = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(xs, off, 64);
      if (lane >= off) xs += y;
    }
    if (lane == 63) wsum[w] = xs;
    __syncthreads();
    int before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (c < tvol) {
      const int e = carry + before + xs - v;
      dm.cell_start[b0 + c] = e;
      dm.cursor[b0 + c] = e;
    }
    carry += tot;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_scatter(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= dm.np) return;
  dm.perm[atomicAdd(&dm.cursor[dm.key[p]], 1)] = p;
}

// The scatter fills each bin in arbitrary order; sorting every bin by the
// original index makes the result the stable counting sort.
__global__ void __launch_bounds__(kBlock) k_cellsort(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= dm.nk) return;
  int *perm = dm.perm;
  const int s = dm.cell_start[k], e = dm.cell_start[k + 1];
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

// Storage order inside a tile: slot-major.  The particles of a tile are laid
// out slot by slot, the first particle (in stable bin order) of every
// non-empty cell in cell order, then the second, and so on; lperm[q] is the
// pre-sort index of the particle stored at q.  Consecutive particles, hence
// the lanes of a wave, then lie in distinct cells, so the node updates of one
// wave-wide LDS atomic never address the same word, while every particle
// array is still read contiguously.  One workgroup per tile; the rank of a
// cell among the cells that hold a slot-j particle comes from wave ballots.
__global__ void __launch_bounds__(kBlock) k_slot_layout(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  const TileGeom &tg = dm.tg;
  if (!*dm.active || (int)blockIdx.x >= tg.ntiles) return;
  const int tvol = tg.tvol;
  const int *cs = dm.cell_start + (size_t)blockIdx.x * tvol;
  const int p0 = cs[0];
  if (p0 == cs[tvol]) return;
  __shared__ int wtot[kBlock / 64];
  __shared__ int wmax[kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int mx = 0;
  for (int c = threadIdx.x; c < tvol; c += kBlock) mx = max(mx, cs[c + 1] - cs[c]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) wmax[w] = mx;
  __syncthreads();
  mx = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
  int dst = p0;  // first position of slot j
  for (int j = 0; j < mx; ++j) {
    for (int c0 = 0; c0 < tvol; c0 += kBlock) {
      const int c = c0 + threadIdx.x;
      const bool has = c < tvol && cs[c + 1] - cs[c] > j;
      const unsigned long long bal = __ballot(has);
      if (lane == 0) wtot[w] = __popcll(bal);
      __syncthreads();
      int before = 0;
      for (int k = 0; k < w; ++k) before += wtot[k];
      const int tot = wtot[0] + wtot[1] + wtot[2] + wtot[3];
      if (has) dm.lperm[dst + before + __popcll(bal & ((1ull << lane) - 1ull))] = dm.perm[cs[c] + j];
      dst += tot;
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_flip(const DomDesc *dd, int ndom) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;
  if (i < ndom && *dd[i].active) *dd[i].cur ^= 1;
}

// Fine-state store / restore (Eq. store_states): to_store = 1 copies the
// current buffer to the store, 0 copies it back.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_copy_state(const DomDesc *dd, int to_store) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= dm.np) return;
  const PartPtrs &cb = dm.pb[*dm.cur];
  const PartPtrs &a = to_store ? cb : dm.st;
  const PartPtrs &b = to_store ? dm.st : cb;
  const int64_t cap = dm.cap;
#pragma unroll
  for (int r = 0; r < D; ++r) {
    b.x[r * cap + p] = a.x[r * cap + p];
    static_cast<TB *>(b.v)[r * cap + p] = static_cast<const TB *>(a.v)[r * cap + p];
  }
#pragma unroll
  for (int r = 0; r < D * D; ++r) {
    static_cast<TB *>(b.B)[r * cap + p] = static_cast<const TB *>(a.B)[r * cap + p];
    static_cast<TB *>(b.F)[r * cap + p] = static_cast<const TB *>(a.F)[r * cap + p];
  }
  b.mass[p] = a.mass[p];
  b.vol[p] = a.vol[p];
  b.mat[p] = a.mat[p];
  b.id[p] = a.id[p];
  b.flags[p] = a.flags[p];
}

// ====================================================================== tiles
// The live tile that workgroup b of a tile launch takes (its slot of the
// live-tile list), its particle range and node-region origin; false for an
// idle slot, so that workgroups without a tile leave after one load.
__device__ inline bool tile_slot(const TileSlot *tl, const TileGeom &tg, int b, int &p0, int &p1, int *org) {
  if (b >= tg.nblocks) return false;
  const int *e = reinterpret_cast<const int *>(tl + b);
  const int t = uload(e);
  p0 = uload(e + 1);
  p1 = uload(e + 2);
  if (t < 0 || p0 >= p1) return false;
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
template <int D, typename T>
__device__ inline bool local_base(const TileGeom &tg, const Stencil<D, T> &st, const int *org, int *l) {
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
// The weights N and the mass terms m_p N are evaluated in FP64 and rounded
// to the bulk type TB (so the active set m_i > 0 and the fixed-point masses
// follow their definitions exactly); the momentum terms are evaluated in TB
// from the TB velocities and affine matrices.  Tile sums are accumulated in
// FP64 LDS (ds_add_f64, which measures about twice as fast as ds_add_f32 on
// gfx950) and added to the FP64 grid.
// kQ (the launches that also select node sets) is a template parameter so
// that the common launch carries no per-node branches; particles of scene
// groups, which are few, add their group masses in a pass of their own.
// The kernel also completes the binning: it reads each particle's arrays
// from the buffer in pre-sort order at lperm[p] and writes them to the other
// buffer at their storage position p, so every array is read once for both
// the permuted copy and the scatter (the host flips the current buffer
// after the launch).
template <int D, typename TB, bool kQ>
__global__ void __launch_bounds__(kBlock) k_p2g(const DomDesc *dd, int *err) {
  constexpr int want_q = kQ ? 1 : 0;
  const DomDesc &dm = dd[blockIdx.y];
  if ((int)blockIdx.x >= dm.tg.nblocks || !*dm.active) return;
  extern __shared__ double lds[];
  // Descriptor fields are copied to registers: the loops below issue
  // atomics, after which the compiler would otherwise reload every field
  // from the descriptor in global memory (a dependent round trip per
  // particle).
  const TileGeom tg = dm.tg;
  const GridDev g = dm.g;
  int p0, p1, org[3];
  if (!tile_slot(dm.tl, tg, blockIdx.x, p0, p1, org)) return;
  const int cur = *dm.cur;
  const PartPtrs P = dm.pb[cur];      // pre-sort order (read at lperm)
  const PartPtrs Q = dm.pb[cur ^ 1];  // storage order (written)
  const int *const lperm = dm.lperm;
  const double scale = dm.scale;
  double *const gm = dm.m;
  double *const gvn = dm.vn;
  long long *const gq_all = dm.q_all;
  long long *const gqg = dm.qg;
  const int64_t cap = dm.cap;
  const TB *v = static_cast<const TB *>(P.v);
  const TB *B = static_cast<const TB *>(P.B);
  const TB *Fs = static_cast<const TB *>(P.F);
  TB *const vd = static_cast<TB *>(Q.v);
  TB *const Bd = static_cast<TB *>(Q.B);
  TB *const Fd = static_cast<TB *>(Q.F);
  const int nreg = tg.nreg;
  const int n_groups = dm.bc.n_groups;
  long long *lq = reinterpret_cast<long long *>(lds);
  double *lm = reinterpret_cast<double *>(lq + (size_t)(1 + kMaxGroups) * nreg);
  double *lmv = lm + nreg;
  const int nq = want_q ? 1 + n_groups : 0;
  for (int r = threadIdx.x; r < nreg * (1 + D); r += kBlock) lm[r] = 0.0;
  for (int r = threadIdx.x; r < nreg * nq; r += kBlock) lq[r] = 0;
  __syncthreads();
  const TB dx_t = (TB)g.dx, Dinv_t = (TB)dm.Dinv;
  int q_next = (p0 + (int)threadIdx.x < p1) ? gload(lperm, p0 + (int)threadIdx.x) : 0;
  for (int p = p0 + threadIdx.x; p < p1; p += kBlock) {
    // the source index of the next particle is fetched one iteration ahead;
    // all of this particle's loads are issued together, one round trip
    const int q = q_next;
    if (p + kBlock < p1) q_next = gload(lperm, p + kBlock);
    double xp[D];
    TB vp[D], Bp[D * D], Fp[D * D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      xp[a] = gload(P.x, a * cap + q);
      vp[a] = gload(v, a * cap + q);
    }
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
      Bp[k] = gload(B, k * cap + q);
      Fp[k] = gload(Fs, k * cap + q);
    }
    const double mp = gload(P.mass, q);
    const double vol = gload(P.vol, q);
    const int mat = gload(P.mat, q);
    const int id = gload(P.id, q);
    const uint8_t fl = gload(P.flags, q);
    // the permuted copy at the storage position
#pragma unroll
    for (int a = 0; a < D; ++a) {
      gstore(Q.x, a * cap + p, xp[a]);
      gstore(vd, a * cap + p, vp[a]);
    }
#pragma unroll
    for (int k = 0; k < D * D; ++k) {
      gstore(Bd, k * cap + p, Bp[k]);
      gstore(Fd, k * cap + p, Fp[k]);
    }
    gstore(Q.mass, p, mp);
    gstore(Q.vol, p, vol);
    gstore(Q.mat, p, mat);
    gstore(Q.id, p, id);
    gstore(Q.flags, p, fl);
    Stencil<D> st;
    stencil_eval<D>(xp, g, st);
    int l[3];
    if (!local_base<D>(tg, st, org, l)) {
      atomicOr(err, kErrTile);
      continue;
    }
    const double mq = mp * scale;
    TB f_t[D];
#pragma unroll
    for (int a = 0; a < D; ++a) f_t[a] = (TB)st.f[a];
#pragma unroll
    for (int s = 0; s < stencil_count<D>(); ++s) {
      int k[3];
      stencil_offset<D>(s, k);
      // N and the mass term in FP64, so that m_i > 0 (the active set) and
      // the fixed-point masses match their definition exactly; the momentum
      // term in the bulk type
      const double N = stencil_N<D>(st, k);
      const int r = region_slot<D>(tg, l, k);
      const TB mN = (TB)(mp * N);
      atomicAdd(&lm[r], (double)mN);
      TB dxv[D];
#pragma unroll
      for (int a = 0; a < D; ++a) dxv[a] = ((TB)k[a] - f_t[a]) * dx_t;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        TB aff = TB(0);
#pragma unroll
        for (int b = 0; b < D; ++b) aff += Bp[a * D + b] * dxv[b];
        atomicAdd(&lmv[a * nreg + r], (double)(mN * (vp[a] + Dinv_t * aff)));
      }
      if constexpr (kQ) {
        const long long q = fixed_mass(N, mq);
        atomicAdd(reinterpret_cast<unsigned long long *>(&lq[r]), (unsigned long long)q);
      }
    }
    if constexpr (kQ) {
      const unsigned gmask = (fl >> 1) & ((1u << n_groups) - 1u);
      if (gmask) {
#pragma unroll
        for (int s = 0; s < stencil_count<D>(); ++s) {
          int k[3];
          stencil_offset<D>(s, k);
          const long long q = fixed_mass(stencil_N<D>(st, k), mq);
          const int r = region_slot<D>(tg, l, k);
          for (int gi = 0; gi < n_groups; ++gi)
            if (gmask & (1u << gi))
              atomicAdd(reinterpret_cast<unsigned long long *>(&lq[(1 + gi) * nreg + r]), (unsigned long long)q);
        }
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
      for (int a = 0; a < D; ++a) atomicAdd(&gvn[i * D + a], lmv[a * nreg + r]);
    }
    if (want_q) {
      if (lq[r] != 0) atomicAdd(reinterpret_cast<unsigned long long *>(&gq_all[i]), (unsigned long long)lq[r]);
      for (int gi = 0; gi < n_groups; ++gi) {
        const long long q = lq[(1 + gi) * nreg + r];
        if (q != 0)
          atomicAdd(reinterpret_cast<unsigned long long *>(&gqg[(int64_t)gi * g.nn + i]), (unsigned long long)q);
      }
    }
  }
}

// v_i = (mv)_i / m_i on active nodes; scene-BC group of each DOF (lowest
// group selecting the node whose mask holds the component); the count of
// active nodes of each block of 256 nodes (k_node_list, which follows, forms
// the total).
template <int D>
__global__ void __launch_bounds__(kBlock) k_p2g_final(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double m = (i < dm.g.nn) ? dm.m[i] : 0.0;
  const unsigned long long act = __ballot(m > 0.0);
  __shared__ int wc[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = (int)__popcll(act);
  __syncthreads();
  if (threadIdx.x == 0 && (int)blockIdx.x < (dm.g.nn + kBlock - 1) / kBlock)
    dm.ncnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
  if (i >= dm.g.nn) return;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    if (m > 0.0) dm.vn[i * D + a] /= m;
    int8_t gsel = -1;
    if (m > 0.0) {
      for (int gi = 0; gi < dm.bc.n_groups; ++gi) {
        if (((dm.bc.mask[gi] >> a) & 1) && dm.qg[(int64_t)gi * dm.g.nn + i] > dm.tau_q) {
          gsel = (int8_t)gi;
          break;
        }
      }
    }
    dm.bcg[i * D + a] = gsel;
  }
}

// ====================================================================== G2P
// APIC G2P with v_i = u_i / dt (Eqs. g2p_v, g2p_B), F <- (I + sum u_i gradN^T) F
// (Eq. F_update) and x <- x + dt v_p (Eq. advection).  Weights and the sums
// v_p, B_p, G = sum u_i gradN^T are formed in the bulk type TB (FP32 in the
// mixed path); v, B and H = F - I are stored in TB, and the update of H and
// the advection of x are carried out in FP64.  The update is applied to H as
// H <- H + G + G H, which equals (I + G)(I + H) - I.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_g2p(const DomDesc *dd, double dt, int *err) {
  const DomDesc &dm = dd[blockIdx.y];
  // workgroups past the domain's particles leave on the descriptor alone;
  // then the launch-uniform flags in one round of scalar loads, then the
  // particle arrays' pointers; data through global-address-space accesses
  if ((int)(blockIdx.x * blockDim.x) >= dm.np) return;
  const int act = uload(dm.active);
  const int cur = uload(dm.cur);
  if (!act) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= dm.np) return;
  const PartPtrs &P = dm.pb[cur];
  const int64_t cap = dm.cap;
  const GridDev g = dm.g;
  double *const px = P.x;
  TB *const v = static_cast<TB *>(P.v);
  TB *const B = static_cast<TB *>(P.B);
  TB *const H = static_cast<TB *>(P.F);
  const double *const gu = dm.u;
  // In 2D, x and H = F - I are loaded together (H is not needed until after
  // the gather, but a load issued there is one more round trip).  In 3D, H
  // is loaded after the gather: holding its nine values through the 27-node
  // gather costs a wave per SIMD, which measures slower.
  constexpr bool kEarlyH = (D == 2);
  double xp[D], Hp[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a) xp[a] = gload((const double *)px, a * cap + p);
  if constexpr (kEarlyH) {
#pragma unroll
    for (int k = 0; k < D * D; ++k) Hp[k] = (double)gload((const TB *)H, k * cap + p);
  }
  Stencil<D, TB> st;
  if (!stencil_eval<D>(xp, g, st)) atomicOr(err, kErrOutOfGrid);
  TB vp[D], Bp[D * D], G[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a) vp[a] = TB(0);
#pragma unroll
  for (int k = 0; k < D * D; ++k) {
    Bp[k] = TB(0);
    G[k] = TB(0);
  }
  const double idt = 1.0 / dt;
  const TB dx_t = (TB)g.dx;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int i = node_flat<D>(g, idx);
    // inactive nodes (m = 0) contribute nothing: the solve that precedes
    // every G2P sets u to zero there (its initial iterate) and its steps
    // change active DOFs only, so no mass test is needed
    const TB N = stencil_N<D>(st, k);
    TB gN[D], dxv[D];
    double ui[D];
    stencil_gradN<D>(st, k, gN);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      dxv[a] = ((TB)k[a] - st.f[a]) * dx_t;
      ui[a] = gload(gu, (int64_t)i * D + a);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const TB vi = (TB)(ui[a] * idt);
      vp[a] += N * vi;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        Bp[a * D + b] += N * vi * dxv[b];
        G[a * D + b] += (TB)ui[a] * gN[b];
      }
    }
  }
  if constexpr (!kEarlyH) {
#pragma unroll
    for (int k = 0; k < D * D; ++k) Hp[k] = (double)gload((const TB *)H, k * cap + p);
  }
  double Hn[D * D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double t = Hp[a * D + b] + (double)G[a * D + b];
#pragma unroll
      for (int e = 0; e < D; ++e) t += (double)G[a * D + e] * Hp[e * D + b];
      Hn[a * D + b] = t;
    }
#pragma unroll
  for (int k = 0; k < D * D; ++k) {
    gstore(H, k * cap + p, (TB)Hn[k]);
    gstore(B, k * cap + p, Bp[k]);
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    gstore(v, a * cap + p, vp[a]);
    gstore(px, a * cap + p, xp[a] + dt * (double)vp[a]);
  }
}

// Elastoplastic materials, after G2P on a domain with a yielding material:
// each particle's elastic F = I + H projected onto the yield set in FP64
// (von_mises_project).  A kernel of its own, so that G2P keeps the registers
// of the elastic update alone (the projection's eigensolve in G2P held 3D
// G2P to two waves per SIMD: fold fine 37.5 -> 25-27 us without it).
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_plastic_return(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if ((int)(blockIdx.x * blockDim.x) >= dm.np) return;
  const int act = uload(dm.active);
  const int plastic = uload(&dm.plastic);
  const int cur = uload(dm.cur);
  if (!act || !plastic) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= dm.np) return;
  const PartPtrs &P = dm.pb[cur];
  const int64_t cap = dm.cap;
  TB *const H = static_cast<TB *>(P.F);
  const int mt = gload((const int *)P.mat, p);
  double Fe[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) Fe[k] = (double)gload((const TB *)H, k * cap + p) + ((k % (D + 1) == 0) ? 1.0 : 0.0);
  if (von_mises_project<D>(Fe, dm.mu[mt], dm.tau_y[mt])) {
#pragma unroll
    for (int k = 0; k < D * D; ++k) gstore(H, k * cap + p, (TB)(Fe[k] - ((k % (D + 1) == 0) ? 1.0 : 0.0)));
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
// Schwarz receiver -> dt * v_bc (work buffer vbc_buf); free -> dt * v^n.
// Clears the gradient and
// the Jacobi-diagonal scatter targets of the first Newton iteration; partial
// sums of the node mass (part_a) for the Newton tolerance floor.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_bc_init(const DomDesc *dd, double dt, int use_schwarz, int vbc_buf,
                                                    int warm_slot) {
  const DomDesc &dm = dd[blockIdx.y];
  const int nb = node_blocks(dm.ndof);
  if (!*dm.active || (int)blockIdx.x >= nb) return;
  __shared__ double red[kBlock / 64];
  const GridDev &g = dm.g;
  TB *gdiag = static_cast<TB *>(dm.gd);
  const double *vbc = wbuf(dm, vbc_buf);
  // warm start: the same solve's displacement in the previous Schwarz
  // iteration, on nodes that were active in that iteration's grid
  const double *wu = (warm_slot >= 0 && dm.warm) ? dm.warm + (size_t)warm_slot * dm.warm_stride : nullptr;
  const double *wm = wu ? wu + dm.ndof : nullptr;
  double msum = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.nn; i += nb * kBlock) {
    const double m = dm.m[i];
    const bool act = m > 0.0;
    if (act) msum += m;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = i * D + a;
      uint8_t f = 0;
      double val = 0.0;
      if (act) {
        const int gi = dm.bcg[k];
        if (gi >= 0) {
          val = scene_value<D>(dm.bc, gi, g, i, a, dt);
        } else if (use_schwarz && dm.recv[i]) {
          val = dt * vbc[k];
        } else {
          f = 1;
          val = (wu && wm[i] > 0.0) ? wu[k] : dt * dm.vn[k];
        }
      }
      dm.fr[k] = f;
      dm.u[k] = val;
      dm.gg[k] = 0.0;
      gdiag[k] = TB(0);
    }
  }
  const double t = block_sum(msum, red);
  if (threadIdx.x == 0) dm.part_a[blockIdx.x] = t;
}

// Solve state at the start of an implicit solve: the gradient scale of the
// absolute Newton floor, sum_i m_i * dx / dt^2.  One workgroup per domain.
__global__ void __launch_bounds__(kBlock) k_solve_begin(const DomDesc *dd, double dt, int warm_slot) {
  const DomDesc &dm = dd[blockIdx.y];
  __shared__ double red[kBlock / 64];
  const bool act = *dm.active != 0;
  const double mtot = act ? reduce_partials(dm.part_a, node_blocks(dm.ndof), red) : 0.0;
  if (threadIdx.x == 0) {
    SolveState &s = *dm.ss;
    s.gref = (act && warm_slot >= 0 && dm.warm)
                 ? dm.warm[(size_t)warm_slot * dm.warm_stride + dm.ndof + dm.g.nn]
                 : -1.0;
    s.gnorm0 = 0.0;
    s.gnorm = 0.0;
    s.gscale = mtot * dm.g.dx / (dt * dt);
    s.alpha = 0.0;
    s.dE = 0.0;
    s.it = 0;
    s.phase = act ? kPhaseGrad : kPhaseDone;
    s.ls_count = 0;
    s.converged = 0;
    s.ls_failed = 0;
    s.newton_iters = 0;
    s.cg_iters = 0;
    s.ls_halvings = 0;
    dm.cg->done = 1;
    dm.cg->iter = 0;
  }
}

// After a solve: its displacement and node masses into warm-start slot
// `slot`; at the frame's first Schwarz iteration (first = 1) also the
// solve's initial gradient norm, the reference of the later iterations'
// Newton tests.
__global__ void __launch_bounds__(kBlock) k_warm_keep(const DomDesc *dd, int slot, int first) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active || !dm.warm) return;
  double *w = dm.warm + (size_t)slot * dm.warm_stride;
  const int stride = gridDim.x * blockDim.x;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = i0; k < dm.ndof; k += stride) w[k] = dm.u[k];
  for (int i = i0; i < dm.g.nn; i += stride) w[dm.ndof + i] = dm.m[i];
  if (first && i0 == 0) w[dm.ndof + dm.g.nn] = dm.ss->gnorm0;
}

// After a solve: its counts added to the domain's running totals (reset = 1
// clears them instead).  One thread per domain.
__global__ void __launch_bounds__(kBlock) k_solve_tally(const DomDesc *dd, int reset) {
  const DomDesc &dm = dd[blockIdx.y];
  if (threadIdx.x != 0) return;
  SolveState &s = *dm.ss;
  if (reset) {
    for (int k = 0; k < 5; ++k) s.tally[k] = 0;
    return;
  }
  if (!*dm.active) return;
  s.tally[0] += s.newton_iters;
  s.tally[1] += s.cg_iters;
  s.tally[2] += s.ls_halvings;
  s.tally[3] += s.converged ? 0 : 1;
  s.tally[4] += s.ls_failed;
}

// ====================================================================== gradient + Hessian
// Per particle at the iterate u: F = (I + sum u_i gradN_i^T) F^n and P(F) in
// FP64; the gradient V P F^nT gradN_i is scattered (FP64).  The particle's
// tangent A = dP/dF (PSD-projected when asked), folded with F^n and V,
// Atil = V C^T A C with C: G -> G F^n, is evaluated in the bulk type TB from
// the analytic eigensystem of the Neo-Hookean Hessian, stored packed, and
// its contribution to the Jacobi diagonal is scattered.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock, 2) k_grad_hess(const DomDesc *dd, int project, int *err) {
  constexpr int n = D * D;
  constexpr int ns = n * (n + 1) / 2;
  const DomDesc &dm = dd[blockIdx.y];
  // workgroups past the domain's tile slots leave on the descriptor alone;
  // then the launch-uniform flags in one round of scalar loads; data through
  // global-address-space accesses
  if ((int)blockIdx.x >= dm.tg.nblocks) return;
  const int act = uload(dm.active);
  const int phase = uload(&dm.ss->phase);
  const int cur = uload(dm.cur);
  const double salpha = gload(&dm.ss->alpha, 0);
  const TileGeom tg = dm.tg;
  if (!act || !phase_wants_grad(phase) || (int)blockIdx.x >= tg.nblocks) return;
  // an accepted line-search step is applied here as u + alpha del (the node
  // kernel that follows stores it, with the same fused multiply-add)
  const bool step = phase == kPhaseStep;
  extern __shared__ double lds[];
  const GridDev g = dm.g;
  int p0, p1, org[3];
  if (!tile_slot(dm.tl, tg, blockIdx.x, p0, p1, org)) return;
  const PartPtrs &P = dm.pb[cur];
  const int64_t cap = dm.cap;
  const double *const px = P.x;
  const TB *const F = static_cast<const TB *>(P.F);
  const int *const pmat = P.mat;
  const double *const pvol = P.vol;
  const double *const gmu = dm.mu, *const glam = dm.lam;
  const double *const gu = dm.u;
  const TB *const gdel = static_cast<const TB *>(dm.del);
  double *const ggr = dm.gg;
  TB *const Atil = static_cast<TB *>(dm.Atil);
  TB *const gdiag = static_cast<TB *>(dm.gd);
  const int nreg = tg.nreg;
  double *lu = lds;
  double *lg = lds + D * nreg;
  double *ld = lds + 2 * D * nreg;
  for (int r = threadIdx.x; r < nreg; r += kBlock) {
    const int i = region_node<D>(tg, g, org, r);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double uv = 0.0;
      if (i >= 0) {
        uv = gload(gu, (int64_t)i * D + a);
        if (step) uv = __builtin_fma(salpha, (double)gload(gdel, (int64_t)i * D + a), uv);
      }
      lu[a * nreg + r] = uv;
      lg[a * nreg + r] = 0.0;
      ld[a * nreg + r] = 0.0;
    }
  }
  __syncthreads();
  for (int p = p0 + threadIdx.x; p < p1; p += kBlock) {
    // the particle's loads together: position, F^n (as H), material, volume;
    // then the material's moduli
    double xp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = gload(px, a * cap + p);
    TB Hn[n];
#pragma unroll
    for (int k = 0; k < n; ++k) Hn[k] = gload(F, k * cap + p);
    const int mt = gload(pmat, p);
    const double V = gload(pvol, p);
    const double mu = gload(gmu, mt), lam = gload(glam, mt);
    // an empty asm that consumes the loaded values keeps the compiler from
    // issuing the loads only after the tile check (one more round trip)
    if constexpr (D == 2)
      asm volatile("" ::"v"(xp[0]), "v"(xp[1]), "v"(Hn[0]), "v"(Hn[1]), "v"(Hn[2]), "v"(Hn[3]), "v"(V), "v"(mu),
                   "v"(lam));
    else
      asm volatile("" ::"v"(xp[0]), "v"(xp[1]), "v"(xp[2]), "v"(Hn[0]), "v"(Hn[1]), "v"(Hn[2]), "v"(Hn[3]),
                   "v"(Hn[4]), "v"(Hn[5]), "v"(Hn[6]), "v"(Hn[7]), "v"(Hn[8]), "v"(V), "v"(mu), "v"(lam));
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
      Fn[k] = (double)Hn[k] + ((k % (D + 1) == 0) ? 1.0 : 0.0);  // F = I + H
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
    double Pk[n];
    if (!nh_stress<D, double>(Fc, mu, lam, Pk, nullptr)) {
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
        for (int c = 0; c < D; ++c) tv += Pk[a * D + c] * Fn[b * D + c];
        T[a * D + b] = V * tv;
      }
    // gradient scatter first, so that T is dead during the tangent work
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
    }
    TB At[ns];
    {
      TB Fb[n], Fnb[n];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        Fb[k] = (TB)Fc[k];
        Fnb[k] = (TB)Fn[k];
      }
      // folded (and, when asked, PSD-projected) tangent from the analytic
      // eigensystem of the Neo-Hookean Hessian
      nh_folded_tangent<D, TB>(Fb, Fnb, (TB)mu, (TB)lam, (TB)V, project != 0, At);
#pragma unroll
      for (int k = 0; k < ns; ++k) gstore(Atil, k * cap + p, At[k]);
    }
    // In 3D, evaluate the stencil again for the diagonal rather than keep its
    // weights (18 doubles) live across the tangent work: an empty register
    // barrier on the position stops the compiler from reusing the first one.
    if constexpr (D == 3) {
#pragma unroll
      for (int a = 0; a < D; ++a) asm volatile("" : "+v"(xp[a]));
      stencil_eval<D>(xp, g, st);
    }
#pragma unroll
    for (int s = 0; s < stencil_count<D>(); ++s) {
      int k[3];
      stencil_offset<D>(s, k);
      double gN[D];
      stencil_gradN<D>(st, k, gN);
      const int r = region_slot<D>(tg, l, k);
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
  __syncthreads();
  for (int r = threadIdx.x; r < nreg; r += kBlock) {
    const int i = region_node<D>(tg, g, org, r);
    if (i < 0) continue;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double gv = lg[a * nreg + r];
      if (gv != 0.0) gatomic_add(ggr, (int64_t)i * D + a, gv);
      const double dv = ld[a * nreg + r];
      if (dv != 0.0) gatomic_add(gdiag, (int64_t)i * D + a, (TB)dv);
    }
  }
}

// Node part of the gradient: + m/dt^2 (u - dt v^n) - m g on active nodes,
// masked to free DOFs; partial |g|^2 (part_a).  The Jacobi diagonal becomes
// scatter + m/dt^2 (1 on non-free DOFs).
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_grad_node(const DomDesc *dd, double dt, double gx, double gy, double gz) {
  const DomDesc &dm = dd[blockIdx.y];
  const int nb = node_blocks(dm.ndof);
  if (!*dm.active || !phase_wants_grad(dm.ss->phase) || (int)blockIdx.x >= nb) return;
  __shared__ double red[kBlock / 64];
  TB *gdiag = static_cast<TB *>(dm.gd);
  // an accepted line-search step: u += alpha del (as the tangent kernel read it)
  const bool step = dm.ss->phase == kPhaseStep;
  const double alpha = step ? dm.ss->alpha : 0.0;
  const TB *del = static_cast<const TB *>(dm.del);
  const double grav[3] = {gx, gy, gz};
  const double idt2 = 1.0 / (dt * dt);
  double s2 = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < dm.g.nn; i += nb * kBlock) {
    const double m = dm.m[i];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = i * D + a;
      double uk = dm.u[k];
      if (step) {
        uk = __builtin_fma(alpha, (double)del[k], uk);
        dm.u[k] = uk;
      }
      double gval = dm.gg[k];
      if (m > 0.0) gval += m * idt2 * (uk - dt * dm.vn[k]) - m * grav[a];
      if (!dm.fr[k]) gval = 0.0;
      dm.gg[k] = gval;
      s2 += gval * gval;
      gdiag[k] = dm.fr[k] ? (TB)((double)gdiag[k] + m * idt2) : TB(1);
    }
  }
  const double t = block_sum(s2, red);
  if (threadIdx.x == 0) dm.part_a[blockIdx.x] = t;
}

// ====================================================================== CG
// Jacobi-preconditioned CG on H del = -g over the free DOFs, in the
// single-reduction form of Chronopoulos and Gear (1989): with u = D^-1 r and
// w = A u, the step length follows from gamma = (r, u) and delta = (w, u)
// alone, alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_(i-1)),
// beta_i = gamma_i / gamma_(i-1), and the direction and its product are
// carried by p_i = u_i + beta_i p_(i-1), s_i = w_i + beta_i s_(i-1).  In exact
// arithmetic the iterates are those of standard PCG.  Both inner products
// are available inside the pass that forms A u (delta through the particles,
// sum_p G:Atil:G + sum_i m_i/dt^2 |u_i|^2), so one launch per iteration
// suffices: kernel boundaries are the only grid-wide barrier, and every
// launch costs one dependent dispatch.
//
// Vectors are stored in the bulk type TB (FP32 in the mixed path); scalars,
// inner products and the vector arithmetic are FP64.

// p = u + beta p_prev, rounded to the storage type.
template <typename TB>
__device__ inline TB cg_direction(TB u, double beta, TB pp) {
#pragma clang fp contract(off)
  const double t = beta * (double)pp;
  return (TB)((double)u + t);
}

// s = w + beta s_old, r = r_old - alpha s, u = r / diag, each rounded to the
// storage type.  No contraction, so the owner of a node and every workgroup
// that recomputes it as a halo node obtain the same bits.
template <typename TB>
__device__ inline void cg_advance(TB r_old, TB w_old, TB s_old, TB dg, double alpha, double beta, TB &s, TB &r,
                                  TB &u) {
#pragma clang fp contract(off)
  const double t = beta * (double)s_old;
  s = (TB)((double)w_old + t);
  const double a = alpha * (double)s;
  r = (TB)((double)r_old - a);
  u = (TB)((double)r / (double)dg);
}

template <typename TB>
__device__ inline TB cg_precond(TB r, TB dg) {
  return (TB)((double)r / (double)dg);
}

__device__ inline void block_sum3(double &a, double &b, double &c, double *lds12) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    lds12[w] = a;
    lds12[4 + w] = b;
    lds12[8 + w] = c;
  }
  __syncthreads();
  a = lds12[0] + lds12[1] + lds12[2] + lds12[3];
  b = lds12[4] + lds12[5] + lds12[6] + lds12[7];
  c = lds12[8] + lds12[9] + lds12[10] + lds12[11];
}

// r_0 = -g, s = p = del = 0, w = 0 on every DOF (r_0 masked to the free
// DOFs); the gradient is cleared for the next Newton iteration and the CG
// state reset.  Runs for domains whose Newton iteration goes on to CG.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_cg_init(const DomDesc *dd, int check, double rtol, double atol,
                                                    int max_newton, double forcing) {
  const DomDesc &dm = dd[blockIdx.y];
  const int nb = node_blocks(dm.ndof);
  if (!*dm.active || (int)blockIdx.x >= nb) return;
  SolveState &st = *dm.ss;
  const int ph = st.phase;
  double eta = 0.0;
  if (check) {
    // The Newton stop test on the fresh gradient, by every workgroup from the
    // same partial sums in the same order: stop when |g_free| <= max(rtol
    // |g_free(u0)|, atol * sum m * dx / dt^2) or after max_newton steps, else
    // go on to CG.  Workgroup 0 records the decision; a workgroup that starts
    // after it did reads the phase it wrote (kPhaseCgInit or kPhaseDone) and
    // reaches the same decision.
    if (!(phase_wants_grad(ph) || ph == kPhaseCgInit)) return;
    __shared__ double red[kBlock / 64];
    const double gn = sqrt(reduce_partials(dm.part_a, nb, red));
    const int it = st.it;
    // a warm-started solve tests against the reference norm of its slot
    const double gn0 = (it == 0) ? (st.gref >= 0.0 ? st.gref : gn) : st.gnorm0;
    const double tol = fmax(rtol * gn0, atol * st.gscale);
    const bool conv = gn <= tol;
    const int next = (conv || it == max_newton) ? kPhaseDone : kPhaseCgInit;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (forcing > 0.0 && next == kPhaseCgInit) {
        // Eisenstat-Walker choice 2 with its safeguards
        if (it == 0) {
          eta = forcing;
        } else {
          const double q = gn / st.gnorm, ep = dm.cg->eta;
          eta = 0.9 * q * q;
          if (0.9 * ep * ep > 0.1) eta = fmax(eta, 0.9 * ep * ep);
        }
        eta = fmin(forcing, fmax(eta, 0.5 * tol / gn));
      }
      if (it == 0) st.gnorm0 = gn0;
      st.gnorm = gn;
      if (conv) st.converged = 1;
      st.phase = next;
    }
    if (next != kPhaseCgInit) return;
  } else if (ph != kPhaseCgInit) {
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CgState &c = *dm.cg;
    c.iter = 0;
    c.done = 0;
    c.eta = eta;
    c.red_cnt = 0;
    c.k_at[0] = 0;
    c.k_at[1] = 0;
  }
  TB *r0 = static_cast<TB *>(dm.cr[0]), *r1 = static_cast<TB *>(dm.cr[1]);
  TB *s0 = static_cast<TB *>(dm.cs[0]), *s1 = static_cast<TB *>(dm.cs[1]);
  TB *w0 = static_cast<TB *>(dm.cw[0]), *w1 = static_cast<TB *>(dm.cw[1]), *w2 = static_cast<TB *>(dm.cw[2]);
  TB *p = static_cast<TB *>(dm.cp), *del = static_cast<TB *>(dm.del);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < dm.ndof; k += nb * kBlock) {
    r0[k] = dm.fr[k] ? (TB)(-dm.gg[k]) : TB(0);
    dm.gg[k] = 0.0;  // scatter target of the next Newton iteration
    r1[k] = TB(0);
    s0[k] = TB(0);
    s1[k] = TB(0);
    w0[k] = TB(0);
    w1[k] = TB(0);
    w2[k] = TB(0);
    p[k] = TB(0);
    del[k] = TB(0);
  }
}

// Scalars of CG launch i from the partial sums (sg, sd, sr) of launch i - 1:
// the stop test on |r_(i-1)| <= rtol |r_0| (or i - 1 = max_cg), beta_(i-1)
// and alpha_(i-1); with write set, the state the next decision needs.
struct CgStep {
  double alpha, beta;
  bool done;
};
// The state launch i reads (written by launches before it): |r_0|^2,
// gamma_(i-1) and alpha_(i-1) of the previous step.
struct CgPrev {
  double rr0, gam, alp;
};
__device__ inline CgPrev cg_prev(const CgState *S, int i) {
  return CgPrev{gload(&S->rr0, 0), gload(&S->gam[i & 1], 0), gload(&S->alp[i & 1], 0)};
}
__device__ inline CgStep cg_scalars(CgState *S, const CgPrev &pv, int i, double sg, double sd, double sr,
                                    double rtol, int max_cg, bool write) {
  CgStep r{0.0, 0.0, false};
  const double rr0 = (i == 1) ? sr : pv.rr0;
  if (i - 1 >= max_cg) {
    r.done = true;
  } else if (i == 1) {
    r.done = !(rr0 > 0.0);
  } else {
    r.done = sqrt(sr) <= rtol * sqrt(rr0);
  }
  if (!r.done) {
    r.beta = (i == 1) ? 0.0 : sg / pv.gam;
    const double den = (i == 1) ? sd : sd - r.beta * sg / pv.alp;
    if (den > 0.0)
      r.alpha = sg / den;
    else
      r.done = true;
  }
  if (write) {
    if (i == 1) S->rr0 = rr0;
    S->gam[(i + 1) & 1] = sg;
    S->alp[(i + 1) & 1] = r.alpha;
  }
  return r;
}

// CG iteration i of a domain (i read from the device state at parity q, so
// launches alternate q = 0, 1 and a chunk of them can be replayed with fixed
// arguments).  For i >= 1 every workgroup sums the partials of launch i - 1
// in the same order and derives the same scalars: the stop test on
// |r_(i-1)| <= rtol |r_0| (or i - 1 = max_cg), beta_(i-1) and alpha_(i-1).
// Owned DOFs then apply p_(i-1) to del and form s_(i-1), r_i, u_i; the tile
// region recomputes u_i at its nodes from r_(i-1), w_(i-1), s_(i-2) in LDS,
// the particles scatter the stiffness part of w_i = A u_i and accumulate
// (w_i, u_i); owned DOFs add the lumped-mass part m_i/dt^2 u_i to w_i and to
// (w_i, u_i), and (r_i, u_i), (r_i, r_i).  i = 0 forms
// u_0 = D^-1 r_0 and w_0 only.  Loads that do not depend on the scalars are
// issued before the reduction.
// split = 1: the scalars are not derived here but read from the state, where
// k_cg_reduce put them after the previous launch (same sums in the same
// order, so both forms give identical results); for launches of many
// workgroups this replaces every workgroup's pass over all partial sums.
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_cg_iter(const DomDesc *dd, int q, double dt, double rtol, int max_cg,
                                                    int split) {
  constexpr int n = D * D;
  constexpr int ns = n * (n + 1) / 2;
  const DomDesc &dm = dd[blockIdx.y];
  // The launch starts in three rounds of scalar loads: the descriptor
  // fields, then every word at an address they give (flags, iteration, the
  // tile's particle range), then the data.  Empty asm statements that consume
  // each round's values keep the compiler from issuing those loads one by one
  // where they are first used (after the early exit), which would chain
  // several more round trips.  The vectors of the rotation are chosen among
  // preloaded pointers instead of indexing the descriptor with the iteration,
  // and data go through global-address-space accesses, so that waiting for
  // them never waits for this wave's LDS atomics as well.
  const TileGeom tg = dm.tg;
  CgState *const S = dm.cg;
  const int *const pactive = dm.active, *const pcur = dm.cur, *const plc = dm.lcnt, *const pnl = dm.nlist;
  const TileSlot *const ptl = dm.tl;
  const uint8_t *const fr = dm.fr;
  const double *const gm = dm.m;
  const TB *const Atil = static_cast<const TB *>(dm.Atil);
  const TB *const dg = static_cast<const TB *>(dm.gd);
  void *const cr0 = dm.cr[0], *const cr1 = dm.cr[1];
  void *const cs0 = dm.cs[0], *const cs1 = dm.cs[1];
  void *const cw0 = dm.cw[0], *const cw1 = dm.cw[1], *const cw2 = dm.cw[2];
  void *const cu = dm.cu, *const cp = dm.cp, *const cdel = dm.del;
  double *const part_cg = dm.part_cg;
  const double *const x0 = dm.pb[0].x, *const x1 = dm.pb[1].x;
  const int ndof = dm.ndof;
  const int pstride = dm.pstride;
  const int64_t cap = dm.cap;
  const GridDev g = dm.g;
  asm volatile("" ::"s"(S), "s"(pactive), "s"(pcur), "s"(plc), "s"(pnl), "s"(ptl), "s"(fr), "s"(gm), "s"(Atil), "s"(dg), "s"(cr0),
               "s"(cs1), "s"(cw0), "s"(cw2), "s"(cu), "s"(cdel), "s"(part_cg), "s"(x0), "s"(x1), "s"(ndof),
               "s"(pstride), "s"(cap), "s"(tg.nblocks), "s"(tg.tvol), "s"(g.n[0]), "s"(g.n[2]), "s"(g.origin[0]),
               "s"(g.inv_dx));
  // workgroups past the domain's tile slots leave on the descriptor alone;
  // the workgroup's slot of the live-tile list and its first active DOF are
  // read with the flags (the node index clamped into the list; used only
  // when valid)
  if ((int)blockIdx.x >= tg.nblocks) return;
  const int tid = threadIdx.x;
  const int bq = (int)blockIdx.x;
  const int j0 = (int)blockIdx.x * kBlock + tid;
  const int act = uload(pactive);
  const int sdone = uload(&S->done);
  const int i = uload(&S->k_at[q]);
  const int cur = uload(pcur);
  const int ntl = uload(plc);
  const int nnl = uload(plc + 1);
  const int *const te4 = reinterpret_cast<const int *>(ptl + bq);  // {tile, p0, p1, pad}, 16-byte aligned
  const int te_t = uload(te4);
  const int te_p0 = uload(te4 + 1);
  const int te_p1 = uload(te4 + 2);
  const int nd0 = gload(pnl, j0 / D < g.nn ? j0 / D : g.nn - 1);
  const double s_rr0 = gload(&S->rr0, 0), s_gam0 = gload(&S->gam[0], 0), s_gam1 = gload(&S->gam[1], 0);
  const double s_alp0 = gload(&S->alp[0], 0), s_alp1 = gload(&S->alp[1], 0);
  const double s_alpha_n = gload(&S->alpha_n, 0), s_beta_n = gload(&S->beta_n, 0);
  const double s_eta = gload(&S->eta, 0);
  asm volatile("" ::"s"(act), "s"(sdone), "s"(i), "s"(cur), "s"(ntl), "s"(nnl), "s"(te_t), "s"(te_p0), "s"(te_p1),
               "v"(nd0));
  const int ndl = nnl * D;  // active DOFs
  const int nbt = cg_work_blocks(ntl, ndl, tg.nblocks);
  if (!act || sdone || (int)blockIdx.x >= nbt) return;
  extern __shared__ double lds[];
  __shared__ double red[12];
  const int i2 = i & 1, i3 = i % 3;
  const TB *const r_old = static_cast<const TB *>(i2 ? cr0 : cr1);  // r_(i-1)
  TB *const r_new = static_cast<TB *>(i2 ? cr1 : cr0);              // r_i
  const TB *const w_old = static_cast<const TB *>(i3 == 0 ? cw2 : (i3 == 1 ? cw0 : cw1));
  TB *const w_new = static_cast<TB *>(i3 == 0 ? cw0 : (i3 == 1 ? cw1 : cw2));
  TB *const w_clr = static_cast<TB *>(i3 == 0 ? cw1 : (i3 == 1 ? cw2 : cw0));
  const TB *const s_old = static_cast<const TB *>(i2 ? cs1 : cs0);
  TB *const s_new = static_cast<TB *>(i2 ? cs0 : cs1);
  TB *const uu = static_cast<TB *>(cu);
  TB *const pp = static_cast<TB *>(cp);
  TB *const del = static_cast<TB *>(cdel);
  const double *const pin = part_cg + (size_t)(q ^ 1) * 3 * pstride;
  double *const pout = part_cg + (size_t)q * 3 * pstride;
  const double *const x = cur ? x1 : x0;
  // scalars of the previous step (launches before this one wrote them)
  const CgPrev prev{s_rr0, i2 ? s_gam1 : s_gam0, i2 ? s_alp1 : s_alp0};
  double alpha = 0.0, beta = 0.0;
  if (i > 0 && split) {
    alpha = s_alpha_n;
    beta = s_beta_n;
  }
  const int p0 = te_p0, p1 = te_p1;
  int org[3] = {0, 0, 0};
  const bool tile_ok = te_t >= 0 && p0 < p1;
  if (tile_ok) tile_origin(tg, te_t, org);
  const int nreg = tg.nreg;
  // --- independent loads
  double sg = 0.0, sd = 0.0, sr = 0.0;
  if (i > 0 && !split)
    for (int j = tid; j < nbt; j += kBlock) {
      sg += gload(pin, j);
      sd += gload(pin, pstride + j);
      sr += gload(pin, 2 * pstride + j);
    }
  int ri = -1;
  TB hr[D], hw[D], hs[D], hd[D];
  uint8_t hf[D];
  if (tile_ok && tid < nreg) {
    ri = region_node<D>(tg, g, org, tid);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = ri * D + a;
      hf[a] = (ri >= 0) ? gload(fr, k) : 0;
      hr[a] = (ri >= 0) ? gload(i == 0 ? (const TB *)r_new : r_old, k) : TB(0);  // r_0 at i = 0
      hw[a] = (ri >= 0 && i > 0) ? gload(w_old, k) : TB(0);
      hs[a] = (ri >= 0 && i > 0) ? gload(s_old, k) : TB(0);
      hd[a] = (ri >= 0) ? gload(dg, k) : TB(1);
    }
  }
  const int pp0 = p0 + tid;
  const bool have_p = tile_ok && pp0 < p1;
  double xp[D];
  TB At[ns];
  if (have_p) {
#pragma unroll
    for (int a = 0; a < D; ++a) xp[a] = gload(x, a * cap + pp0);
#pragma unroll
    for (int k = 0; k < ns; ++k) At[k] = gload(Atil, k * cap + pp0);
  }
  // first owned DOF of the thread (usually its only one): active DOF j0
  const int k0 = (j0 < ndl) ? nd0 * D + j0 % D : -1;
  uint8_t of = 0;
  TB orr = TB(0), ow = TB(0), os = TB(0), od = TB(1), ou = TB(0), op = TB(0), odl = TB(0);
  double om = 0.0;
  if (k0 >= 0) {
    of = gload(fr, k0);
    if (of) {
      orr = gload(i == 0 ? (const TB *)r_new : r_old, k0);
      od = gload(dg, k0);
      om = gload(gm, k0 / D);
      if (i > 0) {
        ow = gload(w_old, k0);
        os = gload(s_old, k0);
        ou = gload((const TB *)uu, k0);
        op = gload((const TB *)pp, k0);
        odl = gload((const TB *)del, k0);
      }
    }
  }
  // --- scalars of iteration i - 1
  if (!split) {
    bool done = false;
    if (i > 0) {
      block_sum3(sg, sd, sr, red);
      const CgStep st = cg_scalars(S, prev, i, sg, sd, sr, fmax(rtol, s_eta), max_cg, blockIdx.x == 0 && tid == 0);
      alpha = st.alpha;
      beta = st.beta;
      done = st.done;
    }
    if (blockIdx.x == 0 && tid == 0) {
      if (done) {
        S->done = 1;
        S->iter = i - 1;
      } else {
        S->iter = i;
        S->k_at[q ^ 1] = i + 1;
      }
    }
    if (done) return;
  }
  const double mdt = 1.0 / (dt * dt);
  double gsum = 0.0, dsum = 0.0, rsum = 0.0;
  // --- owned DOFs: the active DOFs, strided over the working workgroups
  // (only active DOFs ever receive products, so only they need clearing)
  for (int j = j0; j < ndl; j += nbt * kBlock) {
    const bool first = (j == j0);
    const int k = first ? k0 : gload(pnl, j / D) * D + j % D;
    gstore(w_clr, k, TB(0));
    if (!(first ? of : gload(fr, k))) continue;
    TB r, u;
    if (i == 0) {
      r = first ? orr : gload((const TB *)r_new, k);
      u = cg_precond<TB>(r, first ? od : gload(dg, k));
    } else {
      const TB pv = cg_direction<TB>(first ? ou : gload((const TB *)uu, k), beta,
                                     first ? op : gload((const TB *)pp, k));
      gstore(pp, k, pv);
      gstore(del, k, (TB)((double)(first ? odl : gload((const TB *)del, k)) + alpha * (double)pv));
      TB sv;
      if (first)
        cg_advance<TB>(orr, ow, os, od, alpha, beta, sv, r, u);
      else
        cg_advance<TB>(gload(r_old, k), gload(w_old, k), gload(s_old, k), gload(dg, k), alpha, beta, sv, r, u);
      gstore(s_new, k, sv);
      gstore(r_new, k, r);
    }
    gstore(uu, k, u);
    // lumped-mass part of w_i = A u_i; the particle part arrives by atomics
    // from the tiles below, so the owner adds its share atomically too
    const double mu = (first ? om : gload(gm, k / D)) * mdt * (double)u;
    gatomic_add(w_new, k, (TB)mu);
    gsum += (double)r * (double)u;
    rsum += (double)r * (double)r;
    dsum += mu * (double)u;
  }
  // --- w_i = A u_i through the tile's particles
  if (tile_ok) {
    double *lh = lds;
    TB *lu = reinterpret_cast<TB *>(lds + D * nreg);
    for (int r = tid; r < nreg; r += kBlock) {
      const int nd = (r == tid) ? ri : region_node<D>(tg, g, org, r);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        TB u = TB(0);
        if (nd >= 0) {
          const int k = nd * D + a;
          TB fr_r, fw, fs, fd;
          uint8_t ff;
          if (r == tid) {
            ff = hf[a];
            fr_r = hr[a];
            fw = hw[a];
            fs = hs[a];
            fd = hd[a];
          } else {
            ff = gload(fr, k);
            fr_r = gload(i == 0 ? (const TB *)r_new : r_old, k);
            fw = (i > 0) ? gload(w_old, k) : TB(0);
            fs = (i > 0) ? gload(s_old, k) : TB(0);
            fd = gload(dg, k);
          }
          if (ff) {
            if (i == 0) {
              u = cg_precond<TB>(fr_r, fd);
            } else {
              TB s2, r2;
              cg_advance<TB>(fr_r, fw, fs, fd, alpha, beta, s2, r2, u);
            }
          }
        }
        lu[a * nreg + r] = u;
        lh[a * nreg + r] = 0.0;
      }
    }
    __syncthreads();
    for (int p = pp0; p < p1; p += kBlock) {
      if (p != pp0) {
#pragma unroll
        for (int a = 0; a < D; ++a) xp[a] = gload(x, a * cap + p);
#pragma unroll
        for (int k = 0; k < ns; ++k) At[k] = gload(Atil, k * cap + p);
      }
      Stencil<D, TB> st;  // weights in the bulk type
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
        TB gN[D];
        stencil_gradN<D>(st, k, gN);
        const int r = region_slot<D>(tg, l, k);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const TB ua = lu[a * nreg + r];
#pragma unroll
          for (int b = 0; b < D; ++b) G[a * D + b] += ua * gN[b];
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
      dsum += (double)qp;
      // Recompute the weight gradients below instead of keeping all 3^d of
      // them live from the gather: an empty register barrier on the weights.
      if constexpr (D == 3) {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            asm volatile("" : "+v"(st.w[a][c]));
            asm volatile("" : "+v"(st.dw[a][c]));
          }
      }
#pragma unroll
      for (int s = 0; s < stencil_count<D>(); ++s) {
        int k[3];
        stencil_offset<D>(s, k);
        TB gN[D];
        stencil_gradN<D>(st, k, gN);
        const int r = region_slot<D>(tg, l, k);
#pragma unroll
        for (int a = 0; a < D; ++a) {
          TB tv = TB(0);
#pragma unroll
          for (int b = 0; b < D; ++b) tv += T[a * D + b] * gN[b];
          atomicAdd(&lh[a * nreg + r], (double)tv);
        }
      }
    }
    __syncthreads();
    for (int r = tid; r < nreg; r += kBlock) {
      const int nd = (r == tid) ? ri : region_node<D>(tg, g, org, r);
      if (nd < 0) continue;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double hv = lh[a * nreg + r];
        if (hv != 0.0) gatomic_add(w_new, (int64_t)nd * D + a, (TB)hv);
      }
    }
  }
  block_sum3(gsum, dsum, rsum, red);
  if (tid == 0) {
    gstore(pout, blockIdx.x, gsum);
    gstore(pout, pstride + blockIdx.x, dsum);
    gstore(pout, 2 * pstride + blockIdx.x, rsum);
  }
}

// Split mode: after CG launch i of parity q, the launch's partial sums are
// added and the stop test, beta_i and alpha_i derived for launch i + 1.
// Each of the gridDim.x workgroups of a domain adds a contiguous share of the
// partials (lane l taking every 256th, as the fused form does over all of
// them) and stores its three sums in the other parity's partial area, which
// split mode leaves unused until the next CG launch writes it.  The last
// workgroup to arrive (a counter in the CG state, which it resets) adds those
// sums in workgroup order and derives the scalars.  With one workgroup the
// sums are the fused form's.  No workgroup waits for another.
__global__ void __launch_bounds__(kBlock) k_cg_reduce(const DomDesc *dd, int q, double rtol, int max_cg) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  CgState *S = dm.cg;
  if (S->done) return;
  __shared__ double red[12];
  __shared__ int last;
  const int tid = threadIdx.x;
  const int nbt = cg_work_blocks(dm.lcnt[0], dm.lcnt[1] * (dm.ndof / dm.g.nn), dm.tg.nblocks);
  const int nr = gridDim.x;
  const int share = (nbt + nr - 1) / nr;
  const int j0 = blockIdx.x * share;
  const int j1 = min(nbt, j0 + share);
  const int ps = dm.pstride;
  const double *pin = dm.part_cg + (size_t)q * 3 * ps;
  double sg = 0.0, sd = 0.0, sr = 0.0;
  for (int j = j0 + tid; j < j1; j += kBlock) {
    sg += pin[j];
    sd += pin[ps + j];
    sr += pin[2 * ps + j];
  }
  block_sum3(sg, sd, sr, red);
  if (nr > 1) {
    double *tri = dm.part_cg + (size_t)(q ^ 1) * 3 * ps;
    if (tid == 0) {
      __hip_atomic_store(tri + blockIdx.x, sg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(tri + ps + blockIdx.x, sd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(tri + 2 * ps + blockIdx.x, sr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(&S->red_cnt, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == nr - 1;
    }
    __syncthreads();
    if (!last) return;
    sg = sd = sr = 0.0;
    for (int j = tid; j < nr; j += kBlock) {
      sg += __hip_atomic_load(tri + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sd += __hip_atomic_load(tri + ps + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sr += __hip_atomic_load(tri + 2 * ps + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum3(sg, sd, sr, red);
    if (tid == 0) __hip_atomic_store(&S->red_cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (tid == 0) {
    const int n = S->k_at[q] + 1;
    const CgStep st = cg_scalars(S, cg_prev(S, n), n, sg, sd, sr, fmax(rtol, S->eta), max_cg, true);
    S->alpha_n = st.alpha;
    S->beta_n = st.beta;
    if (st.done) {
      S->done = 1;
      S->iter = n - 1;
    } else {
      S->iter = n;
      S->k_at[q ^ 1] = n;
    }
  }
}

// ====================================================================== line search
// A domain evaluates the line search when its CG has finished in this cycle
// (first evaluation, alpha = 1) or when it is already searching (alpha from
// the state).
__device__ inline bool ls_evaluates(const DomDesc &dm, double &alpha) {
  const int ph = dm.ss->phase;
  if (ph == kPhaseLs) {
    alpha = dm.ss->alpha;
    return true;
  }
  if ((ph == kPhaseCgInit || ph == kPhaseCg) && dm.cg->done) {
    alpha = 1.0;
    return true;
  }
  return false;
}

// E(u + alpha del) - E(u) in cancellation-free form, one launch: workgroups
// [0, nbp) take the particles, [nbp, nbp + nbn) the nodes.
// Particle part: V [mu/2 (2 F:Dm + Dm:Dm) - mu L + lam/2 L (2 ln J + L)] with
// L = log1p(dJ / J) and dJ = det(F + Dm) - det F expanded in powers of Dm
// (+inf on inversion); partials in part_b.  Node part:
// m/(2 dt^2) (2 alpha (u - dt v^n).del + alpha^2 |del|^2) - alpha m g.del;
// partials in part_a.  The node workgroups also clear the Jacobi-diagonal
// scatter target for the next Newton iteration (CG no longer reads it).
template <int D, typename TB>
__global__ void __launch_bounds__(kBlock) k_delta_energy(const DomDesc *dd, double dt, double gx, double gy, double gz) {
  constexpr int n = D * D;
  const DomDesc &dm = dd[blockIdx.y];
  const int nbp = particle_blocks(dm.np), nbn = node_blocks(dm.ndof);
  double alpha = 0.0;
  if (!*dm.active || (int)blockIdx.x >= nbp + nbn || !ls_evaluates(dm, alpha)) return;
  __shared__ double red[kBlock / 64];
  const GridDev &g = dm.g;
  const TB *del = static_cast<const TB *>(dm.del);
  double e = 0.0;
  if ((int)blockIdx.x < nbp) {
    const PartPtrs &P = dm.pb[*dm.cur];
    const int64_t cap = dm.cap;
    const TB *F = static_cast<const TB *>(P.F);
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < dm.np; p += nbp * kBlock) {
      double xp[D];
#pragma unroll
      for (int a = 0; a < D; ++a) xp[a] = P.x[a * cap + p];
      Stencil<D> st;
      stencil_eval<D>(xp, g, st);
      double Gu[n], Gd[n], Fn[n];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        Gu[k] = 0.0;
        Gd[k] = 0.0;
        Fn[k] = load_F<D>(F, cap, p, k);
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
          const double ua = dm.u[i * D + a], da = (double)del[i * D + a];
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
      const int mt = P.mat[p];
      const double mu = dm.mu[mt], lam = dm.lam[mt];
      e += P.vol[p] * (0.5 * mu * (2.0 * FD + DD) - mu * L + 0.5 * lam * L * (2.0 * lnJ + L));
    }
    const double t = block_sum(e, red);
    if (threadIdx.x == 0) dm.part_b[blockIdx.x] = t;
  } else {
    const int bn = blockIdx.x - nbp;
    const double grav[3] = {gx, gy, gz};
    TB *gdiag = static_cast<TB *>(dm.gd);
    for (int i = bn * blockDim.x + threadIdx.x; i < g.nn; i += nbn * kBlock) {
#pragma unroll
      for (int a = 0; a < D; ++a) gdiag[i * D + a] = TB(0);
      const double m = dm.m[i];
      if (!(m > 0.0)) continue;
      double rd = 0.0, dd2 = 0.0, gd = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double dv = (double)del[i * D + a];
        rd += (dm.u[i * D + a] - dt * dm.vn[i * D + a]) * dv;
        dd2 += dv * dv;
        gd += grav[a] * dv;
      }
      e += m / (2.0 * dt * dt) * (2.0 * alpha * rd + alpha * alpha * dd2) - alpha * m * gd;
    }
    const double t = block_sum(e, red);
    if (threadIdx.x == 0) dm.part_a[bn] = t;
  }
}

// Per-domain decisions after the CG launches of a cycle (one workgroup per
// domain): a freshly initialised CG is now running; a CG that finished starts
// the line search (its iteration count goes to the statistics, and its first
// evaluation at alpha = 1 is the one just computed); a searching domain
// accepts when the energy change is negative, else halves alpha, or gives up
// after max_ls halvings (the iterate is kept and the solve ends).
__global__ void __launch_bounds__(kBlock) k_ls_check(const DomDesc *dd, int max_ls) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  SolveState *s = dm.ss;
  const int ph = s->phase;
  const bool cg_over = (ph == kPhaseCgInit || ph == kPhaseCg) && dm.cg->done;
  if (!cg_over && ph != kPhaseLs) {
    if (ph == kPhaseCgInit && threadIdx.x == 0) s->phase = kPhaseCg;
    return;
  }
  __shared__ double red[kBlock / 64];
  const double en = reduce_partials(dm.part_a, node_blocks(dm.ndof), red);
  const double ep = reduce_partials(dm.part_b, particle_blocks(dm.np), red);
  if (threadIdx.x == 0) {
    if (cg_over) {
      s->cg_iters += dm.cg->iter;
      s->alpha = 1.0;
      s->ls_count = 0;
    }
    const double dE = en + ep;
    s->dE = dE;
    if (dE < 0.0) {
      // u += alpha del is applied by the next gradient pass (the tangent
      // kernel reads u + alpha del, the node kernel stores it)
      s->phase = kPhaseStep;
      s->newton_iters += 1;
      s->it += 1;
    } else if (s->ls_count == max_ls) {
      s->ls_failed = 1;
      s->phase = kPhaseDone;
    } else {
      s->alpha *= 0.5;
      s->ls_count += 1;
      s->ls_halvings += 1;
      s->phase = kPhaseLs;
    }
  }
}

// ====================================================================== interface
// Fixed-point node mass of the boundary-layer particles (Eq. boundary_grid_set).
template <int D>
__global__ void __launch_bounds__(kBlock) k_qbnd(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= dm.np) return;
  const PartPtrs &P = dm.pb[*dm.cur];
  if (!(P.flags[p] & 1u)) return;
  double xp[D];
#pragma unroll
  for (int a = 0; a < D; ++a) xp[a] = P.x[a * dm.cap + p];
  Stencil<D> st;
  stencil_eval<D>(xp, dm.g, st);
  const double mq = P.mass[p] * dm.scale;
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const long long q = fixed_mass(stencil_N<D>(st, k), mq);
    if (q != 0)
      atomicAdd(reinterpret_cast<unsigned long long *>(&dm.q_bnd[node_flat<D>(dm.g, idx)]), (unsigned long long)q);
  }
}

// Boundary node set Gamma (nodes whose boundary-layer mass exceeds tau) and
// the receiver set before arbitration; the fixed-point accumulator is reset
// for the next build.
__global__ void __launch_bounds__(kBlock) k_gamma(const DomDesc *dd) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= dm.g.nn) return;
  const uint8_t gsel = (dm.q_bnd[i] > dm.tau_q && dm.m[i] > 0.0) ? 1 : 0;
  dm.q_bnd[i] = 0;
  dm.gamma[i] = gsel;
  dm.recv[i] = gsel;
}

// Number of receiver nodes of each domain; one workgroup per domain.
__global__ void __launch_bounds__(kBlock) k_count_recv(const DomDesc *dd, int *out) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  __shared__ int red[kBlock / 64];
  // the flags are 0/1 bytes: 16 per thread and step, counted four to a word
  const int nn = dm.g.nn;
  const uint8_t *rv = dm.recv;
  int c = 0;
  for (int i0 = threadIdx.x * 16; i0 < nn; i0 += kBlock * 16) {
    if (i0 + 16 <= nn) {
      const uint4 w = *reinterpret_cast<const uint4 *>(rv + i0);
      c += __popc(w.x) + __popc(w.y) + __popc(w.z) + __popc(w.w);
    } else {
      for (int i = i0; i < nn; ++i) c += rv[i] ? 1 : 0;
    }
  }
  c = block_sum_int(c, red);
  if (threadIdx.x == 0) out[blockIdx.y] = c;
}

// Overlap arbitration (Eq. overlap_donor): a coarse boundary node whose
// lattice point is a fine boundary node is ambiguous; the larger fixed-point
// node mass donates (ties: the coarse side) and leaves its receiver set.
template <int D>
__global__ void __launch_bounds__(kBlock) k_arbitrate(const DomDesc *ddB, const DomDesc *ddS, int *n_amb) {
  const DomDesc &B = ddB[blockIdx.y], &S = ddS[blockIdx.y];
  if (!*B.active) return;
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= B.g.nn || !B.gamma[I]) return;
  int iB[3], jS[3];
  node_unflat<D>(B.g, I, iB);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const long long L = B.g.origin_q[a] + (long long)iB[a] * B.g.dx_q;
    const long long t = L - S.g.origin_q[a];
    if (t < 0 || t % S.g.dx_q != 0 || t / S.g.dx_q >= S.g.n[a]) return;
    jS[a] = (int)(t / S.g.dx_q);
  }
  const int j = node_flat<D>(S.g, jS);
  if (!S.gamma[j]) return;
  atomicAdd(&n_amb[blockIdx.y], 1);
  if (B.q_all[I] >= S.q_all[j])
    B.recv[I] = 0;
  else
    S.recv[j] = 0;
}

__global__ void __launch_bounds__(kBlock) k_zero_proj(const DomDesc *ddB) {
  const DomDesc &B = ddB[blockIdx.y];
  if (!*B.active) return;
  const int stride = gridDim.x * blockDim.x;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < B.ndof; k += stride) B.pnum[k] = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < B.g.nn; i += stride) B.pden[i] = 0.0;
}

// Pi_{S->B} numerator and denominator: every active fine node j scatters
// m_j N_I(x_j) and m_j v_j N_I(x_j) onto its coarse stencil.  The fine field
// is S's P2G velocity unless an external array is given (a batch of one).
template <int D>
__global__ void __launch_bounds__(kBlock) k_project_scatter(const DomDesc *ddS, const DomDesc *ddB, const double *vS_ext, int *err) {
  const DomDesc &S = ddS[blockIdx.y], &B = ddB[blockIdx.y];
  if (!*S.active) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.g.nn) return;
  const double m = S.m[j];
  if (!(m > 0.0)) return;
  const double *vS = vS_ext ? vS_ext : S.vn;
  int jS[3];
  double xj[D];
  node_unflat<D>(S.g, j, jS);
  node_position<D>(S.g, jS, xj);
  Stencil<D> st;
  if (!stencil_eval<D>(xj, B.g, st)) {
    atomicOr(err, kErrOutOfGrid);
    return;
  }
#pragma unroll
  for (int s = 0; s < stencil_count<D>(); ++s) {
    int k[3], idx[3];
    stencil_offset<D>(s, k);
#pragma unroll
    for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
    const int I = node_flat<D>(B.g, idx);
    // only the receivers' sums are read (by the division and its transpose);
    // skipping the others removes most of the contended atomics
    if (!B.recv[I]) continue;
    const double w = m * stencil_N<D>(st, k);
    atomicAdd(&B.pden[I], w);
#pragma unroll
    for (int a = 0; a < D; ++a) atomicAdd(&B.pnum[I * D + a], w * vS[j * D + a]);
  }
}

// out_I = num_I / (den_I + eps_tol) on coarse receivers, 0 elsewhere; out is
// work buffer `which` of B, or out_ext when which < 0.
template <int D>
__global__ void __launch_bounds__(kBlock) k_project_final(const DomDesc *ddB, double eps_tol, int which, double *out_ext) {
  const DomDesc &B = ddB[blockIdx.y];
  if (!*B.active) return;
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= B.g.nn) return;
  double *out = which < 0 ? out_ext : wbuf(B, which);
  const bool rc = B.recv[I];
#pragma unroll
  for (int a = 0; a < D; ++a) out[I * D + a] = rc ? B.pnum[I * D + a] / (B.pden[I] + eps_tol) : 0.0;
}

// I_{B->S} at the fine receivers (Eq. interp_BtoS): source is B's buffer src
// (or vB_ext when src < 0), target S's buffer dst (or out_ext when dst < 0).
template <int D>
__global__ void __launch_bounds__(kBlock) k_interp(const DomDesc *ddB, const DomDesc *ddS, int src, const double *vB_ext, int dst,
                         double *out_ext, int *err) {
  const DomDesc &B = ddB[blockIdx.y], &S = ddS[blockIdx.y];
  if (!*S.active) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.g.nn) return;
  const double *vB = src < 0 ? vB_ext : wbuf(B, src);
  double *out = dst < 0 ? out_ext : wbuf(S, dst);
  double acc[D];
#pragma unroll
  for (int a = 0; a < D; ++a) acc[a] = 0.0;
  if (S.recv[j]) {
    int jS[3];
    double xj[D];
    node_unflat<D>(S.g, j, jS);
    node_position<D>(S.g, jS, xj);
    Stencil<D> st;
    if (!stencil_eval<D>(xj, B.g, st)) {
      atomicOr(err, kErrOutOfGrid);
    } else {
#pragma unroll
      for (int s = 0; s < stencil_count<D>(); ++s) {
        int k[3], idx[3];
        stencil_offset<D>(s, k);
#pragma unroll
        for (int a = 0; a < D; ++a) idx[a] = st.base[a] + k[a];
        const int I = node_flat<D>(B.g, idx);
        if (!(B.m[I] > 0.0)) continue;
        const double N = stencil_N<D>(st, k);
#pragma unroll
        for (int a = 0; a < D; ++a) acc[a] += N * vB[I * D + a];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) out[j * D + a] = acc[a];
}

// T_m (Eq. temporal_interp) into the Schwarz data: v_bc = (1 - am) a + am b
// for work buffers a, b.
template <int D>
__global__ void __launch_bounds__(kBlock) k_temporal(const DomDesc *dd, double am, int a_buf, int b_buf) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const double *a = wbuf(dm, a_buf), *b = wbuf(dm, b_buf);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < dm.ndof; k += gridDim.x * blockDim.x)
    dm.vbc[k] = (1.0 - am) * a[k] + am * b[k];
}

// ---------------------------------------------------------------- refined regions that overlap
// Node of grid G at the lattice point of node i of grid A, or -1.
template <int D>
__device__ inline int coincident_node(const GridDev &A, int i, const GridDev &G) {
  int ia[3], jg[3] = {0, 0, 0};
  node_unflat<D>(A, i, ia);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const long long L = A.origin_q[a] + (long long)ia[a] * A.dx_q;
    const long long t = L - G.origin_q[a];
    if (t < 0 || t % G.dx_q != 0 || t / G.dx_q >= G.n[a]) return -1;
    jg[a] = (int)(t / G.dx_q);
  }
  return node_flat<D>(G, jg);
}

// Arbitration between the n fine domains of a multi group (Eq. overlap_donor
// applied pairwise): a node in the boundary sets of fine domains f and g at
// one lattice point is ambiguous; the side with the larger fixed-point node
// mass donates (ties: the lower index) and leaves its own receiver set.
// Reads boundary sets and masses only, so the order of the pairs does not
// matter; ambiguous pairs are counted once, at the lower index.
template <int D>
__global__ void __launch_bounds__(kBlock) k_fine_arbitrate(const DomDesc *dd, int n, int *n_amb) {
  const int f = blockIdx.y;
  const DomDesc &F = dd[f];
  if (!*F.active) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F.g.nn || !F.gamma[j]) return;
  bool donor = false;
  for (int g = 0; g < n; ++g) {
    if (g == f) continue;
    const DomDesc &G = dd[g];
    const int jg = coincident_node<D>(F.g, j, G.g);
    if (jg < 0 || !G.gamma[jg]) continue;
    if (f < g) atomicAdd(&n_amb[f], 1);
    const long long qf = F.q_all[j], qg = G.q_all[jg];
    if (qf > qg || (qf == qg && f < g)) donor = true;
  }
  if (donor) F.recv[j] = 0;
}

// Links of the fine receivers after all arbitration: a receiver node of f
// lying in another fine domain's material (the coincident node active with
// a fixed-point mass above that domain's threshold) takes its data from the
// one of largest mass (ties: the lower index); flink[j] = {g, node}, or
// {-1, -1} where the coarse domain donates.
template <int D>
__global__ void __launch_bounds__(kBlock) k_fine_links(const DomDesc *dd, int n) {
  const int f = blockIdx.y;
  const DomDesc &F = dd[f];
  if (!*F.active) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F.g.nn) return;
  int bg = -1, bn = -1;
  long long best = 0;
  if (F.recv[j]) {
    for (int g = 0; g < n; ++g) {
      if (g == f) continue;
      const DomDesc &G = dd[g];
      const int jg = coincident_node<D>(F.g, j, G.g);
      if (jg < 0 || !(G.m[jg] > 0.0)) continue;
      const long long q = G.q_all[jg];
      if (q <= G.tau_q) continue;
      if (bg < 0 || q > best) {
        bg = g;
        bn = jg;
        best = q;
      }
    }
  }
  F.flink[2 * j] = bg;
  F.flink[2 * j + 1] = bn;
}

// Linked receivers' data: the donor's grid velocity u / dt of the solve kept
// in its slot `slot` (its node active then), into v_bc (dst_buf < 0) or a
// work buffer.
template <int D>
__global__ void __launch_bounds__(kBlock) k_fine_link_apply(const DomDesc *dd, int slot, double dt, int dst_buf) {
  const DomDesc &F = dd[blockIdx.y];
  if (!*F.active) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F.g.nn) return;
  const int g = F.flink[2 * j];
  if (g < 0) return;
  const int jg = F.flink[2 * j + 1];
  const DomDesc &G = dd[g];
  const double *w = G.warm + (size_t)slot * G.warm_stride;
  if (!(w[G.ndof + jg] > 0.0)) return;
  double *dst = dst_buf < 0 ? F.vbc : wbuf(F, dst_buf);
#pragma unroll
  for (int a = 0; a < D; ++a) dst[j * D + a] = w[(size_t)jg * D + a] / dt;
}

// w2 = u / dt on active nodes, 0 elsewhere (v_B^(k+1) of Eq. implicit_solve_coarse).
template <int D>
__global__ void __launch_bounds__(kBlock) k_vel_from_u(const DomDesc *dd, double dt) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= dm.g.nn) return;
  const bool act = dm.m[i] > 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) dm.w2[i * D + a] = act ? dm.u[i * D + a] / dt : 0.0;
}

// v_bc = work buffer src.
template <int D>
__global__ void __launch_bounds__(kBlock) k_copy_vbc(const DomDesc *dd, int src) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  const double *s = wbuf(dm, src);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < dm.ndof; k += gridDim.x * blockDim.x) dm.vbc[k] = s[k];
}

// Partial sums over receiver nodes of |a - b|^2 and |a|^2 (Eq.
// convergence_residuals) into part_b[2 block], part_b[2 block + 1].
template <int D>
__global__ void __launch_bounds__(kBlock) k_resid(const DomDesc *dd, int a_buf, int b_buf) {
  const DomDesc &dm = dd[blockIdx.y];
  const int nb = node_blocks(dm.g.nn);
  if (!*dm.active || (int)blockIdx.x >= nb) return;
  __shared__ double red[8];
  const double *a = wbuf(dm, a_buf), *b = wbuf(dm, b_buf);
  double s = 0.0, t = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < dm.g.nn; i += nb * kBlock) {
    if (!dm.recv[i]) continue;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double e = a[i * D + c] - b[i * D + c];
      s += e * e;
      t += a[i * D + c] * a[i * D + c];
    }
  }
  block_sum2(s, t, red);
  if (threadIdx.x == 0) {
    dm.part_b[2 * blockIdx.x] = s;
    dm.part_b[2 * blockIdx.x + 1] = t;
  }
}

// Sums of the residual partials of each domain into out[2 y], out[2 y + 1];
// one workgroup per domain.
__global__ void __launch_bounds__(kBlock) k_resid_final(const DomDesc *dd, double *out) {
  const DomDesc &dm = dd[blockIdx.y];
  if (!*dm.active) return;
  __shared__ double red[8];
  const int nb = node_blocks(dm.g.nn);
  double s = 0.0, t = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    s += dm.part_b[2 * i];
    t += dm.part_b[2 * i + 1];
  }
  block_sum2(s, t, red);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.y] = s;
    out[2 * blockIdx.y + 1] = t;
  }
}

// ====================================================================== instantiations
#define OSMPM_INST_D(D)                                                                                  \
  template __global__ void k_keys<D>(const DomDesc *, int *);                                            \
  template __global__ void k_p2g_final<D>(const DomDesc *);                                              \
  template __global__ void k_qbnd<D>(const DomDesc *);                                                   \
  template __global__ void k_arbitrate<D>(const DomDesc *, const DomDesc *, int *);                      \
  template __global__ void k_project_scatter<D>(const DomDesc *, const DomDesc *, const double *, int *); \
  template __global__ void k_project_final<D>(const DomDesc *, double, int, double *);                   \
  template __global__ void k_interp<D>(const DomDesc *, const DomDesc *, int, const double *, int, double *, \
                                       int *);                                                           \
  template __global__ void k_temporal<D>(const DomDesc *, double, int, int);                                       \
  template __global__ void k_vel_from_u<D>(const DomDesc *, double);                                     \
  template __global__ void k_resid<D>(const DomDesc *, int, int);                                        \
  template __global__ void k_fine_arbitrate<D>(const DomDesc *, int, int *);                             \
  template __global__ void k_fine_links<D>(const DomDesc *, int);                                        \
  template __global__ void k_fine_link_apply<D>(const DomDesc *, int, double, int);                      \
  template __global__ void k_copy_vbc<D>(const DomDesc *, int);

#define OSMPM_INST_DT(D, TB)                                                                    \
  template __global__ void k_bc_init<D, TB>(const DomDesc *, double, int, int, int);                      \
  template __global__ void k_copy_state<D, TB>(const DomDesc *, int);                           \
  template __global__ void k_p2g<D, TB, false>(const DomDesc *, int *);                         \
  template __global__ void k_p2g<D, TB, true>(const DomDesc *, int *);                          \
  template __global__ void k_g2p<D, TB>(const DomDesc *, double, int *);                        \
  template __global__ void k_plastic_return<D, TB>(const DomDesc *);                            \
  template __global__ void k_grad_hess<D, TB>(const DomDesc *, int, int *);                     \
  template __global__ void k_grad_node<D, TB>(const DomDesc *, double, double, double, double); \
  template __global__ void k_cg_init<D, TB>(const DomDesc *, int, double, double, int, double);                                   \
  template __global__ void k_cg_iter<D, TB>(const DomDesc *, int, double, double, int, int);    \
  template __global__ void k_delta_energy<D, TB>(const DomDesc *, double, double, double, double);

OSMPM_INST_D(2)
OSMPM_INST_D(3)
OSMPM_INST_DT(2, double)
OSMPM_INST_DT(2, float)
OSMPM_INST_DT(3, double)
OSMPM_INST_DT(3, float)

}  // namespace osmpm
