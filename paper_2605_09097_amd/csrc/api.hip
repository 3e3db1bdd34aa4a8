// Host side of the C ABI declared in include/osmpm.h: handle management,
// the binning/P2G/G2P pipelines, the Newton-PCG-line-search driver of one
// implicit solve and the multiplicative Schwarz frame of Alg. 1.
//
// The host only sequences kernels and reads back a handful of scalars:
// the Newton gradient norm, the CG state once per chunk of iterations, the
// line-search energy change and the Schwarz residuals.  All arithmetic on
// particles and nodes runs in the kernels of kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "../../include/osmpm.h"
#include "kernels.hpp"

using namespace osmpm;

namespace {

constexpr int kCgChunk = 8;

// Particle arrays, component-major [rows][capacity].  Positions, masses and
// volumes are FP64; velocities, affine matrices and deformation gradients
// are stored in the domain's bulk type (FP64, or FP32 in the mixed path).
struct PartBuf {
  double *x = nullptr, *mass = nullptr, *vol = nullptr;
  void *v = nullptr, *B = nullptr, *F = nullptr;
  int *mat = nullptr, *id = nullptr;
  uint8_t *flags = nullptr;
};

int blocks_for(int64_t n, int cap_blocks = 1024) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap_blocks) b = cap_blocks;
  return (int)b;
}

}  // namespace

// Kernel timing: HIP events recorded on the context stream around every
// launch of the instrumented kernels while profiling is enabled.
struct ProfPending {
  hipEvent_t a, b;
  int which;
  double bytes;
  int cg_iter;  // iteration index of a CG launch, -1 otherwise
};
struct ProfSlot {
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0;
};

struct osmpm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int *d_err = nullptr;
  int *d_count = nullptr;  // small device counters (ambiguous nodes)
  double *h_pin = nullptr;
  size_t h_pin_doubles = 0;
  std::string last_error;
  bool prof = false;
  ProfSlot slots[OSMPM_K_COUNT];
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfPending> pending;
};

struct osmpm_domain {
  osmpm_ctx *ctx = nullptr;
  int D = 2;
  osmpm_grid desc{};
  GridDev g{};
  TileGeom tg{};
  int precision = 0;
  int64_t cap = 0;
  int np = 0;
  PartBuf pb[2], st;
  int cur = 0;
  // binning
  int nk = 0;
  int *key = nullptr, *count = nullptr, *cell_start = nullptr, *cursor = nullptr, *perm = nullptr;
  // materials
  int n_mat = 0;
  double *mu = nullptr, *lam = nullptr;
  // node selection
  double m_ref = 1.0, tau = 0.0;
  SceneBC bc{};
  // grid
  double *m = nullptr, *vn = nullptr, *u = nullptr, *vbc = nullptr;
  int8_t *bcg = nullptr;
  uint8_t *gamma = nullptr, *recv = nullptr, *fr = nullptr;
  long long *q_all = nullptr, *q_bnd = nullptr, *qg = nullptr;
  // solver
  double *gg = nullptr;  // Newton gradient (FP64)
  // bulk-type arrays: Jacobi diagonal, CG vectors, per-particle tangents
  void *gd = nullptr, *r = nullptr, *z = nullptr, *p0 = nullptr, *p1 = nullptr, *del = nullptr, *Hp = nullptr,
       *Atil = nullptr;
  size_t tb = sizeof(double);  // bytes of the bulk type
  CgState *cg = nullptr;
  double *part_a = nullptr, *part_b = nullptr, *part_q = nullptr, *part_rz = nullptr, *part_rr = nullptr;
  int nb_node = 1, nb_part = 1;
  int cg_hint = 8;  // CG iterations of the previous solve (first batch size)
  // interface / Schwarz work buffers ([nn][D] unless noted)
  double *pnum = nullptr, *pden = nullptr /*[nn]*/, *w0 = nullptr, *w1 = nullptr, *w2 = nullptr, *w3 = nullptr;
  bool have_p2g = false;
  std::vector<void *> allocs;
};

// ---------------------------------------------------------------- helpers
namespace {

osmpm_status fail(osmpm_ctx *c, osmpm_status s, const std::string &msg) {
  if (c) c->last_error = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                                            \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail((ctx), OSMPM_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
osmpm_status dalloc(osmpm_domain *d, T **p, size_t n) {
  if (n == 0) n = 1;
  void *q = nullptr;
  if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return fail(d->ctx, OSMPM_E_NO_MEMORY, "hipMalloc failed");
  }
  d->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return OSMPM_OK;
}

osmpm_status dalloc_bytes(osmpm_domain *d, void **p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return fail(d->ctx, OSMPM_E_NO_MEMORY, "hipMalloc failed");
  }
  d->allocs.push_back(*p);
  return OSMPM_OK;
}

osmpm_status ensure_pin(osmpm_ctx *c, size_t doubles) {
  if (c->h_pin_doubles >= doubles) return OSMPM_OK;
  if (c->h_pin) (void)hipHostFree(c->h_pin);
  c->h_pin = nullptr;
  size_t n = std::max<size_t>(doubles, 4096);
  if (hipHostMalloc((void **)&c->h_pin, n * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(c, OSMPM_E_NO_MEMORY, "hipHostMalloc failed");
  c->h_pin_doubles = n;
  return OSMPM_OK;
}

// ---------------------------------------------------------------- profiling
hipEvent_t prof_event(osmpm_ctx *c) {
  if (c->ev_pool.empty()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDefault) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = c->ev_pool.back();
  c->ev_pool.pop_back();
  return e;
}

// Launch of an instrumented kernel.  With profiling on, the dispatch itself
// carries the start and stop timestamps (hipExtLaunchKernelGGL), so no extra
// packets are inserted between kernels.
template <typename F, typename... Args>
void launch(osmpm_ctx *c, int which, double bytes, int cg_iter, F kernel, dim3 grid, dim3 block, uint32_t shm,
            Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (c->prof) {
    a = prof_event(c);
    b = prof_event(c);
    if (!a || !b) a = b = nullptr;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, shm, c->stream, a, b, 0, args...);
  if (a) c->pending.push_back({a, b, which, bytes, cg_iter});
}

// Folds completed timings into the counters; call only after the stream has
// been synchronised.  CG launches at or beyond `cg_done` iterations (those
// that found the solve finished and exited) are dropped.
void prof_harvest(osmpm_ctx *c, int cg_done = 1 << 30) {
  for (const ProfPending &p : c->pending) {
    if (p.cg_iter < 0 || p.cg_iter < cg_done) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        ProfSlot &sl = c->slots[p.which];
        sl.launches += 1;
        sl.ms += ms;
        sl.bytes += p.bytes;
      }
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

// Algorithmic bytes of one launch: the data the operation must move once
// (particle arrays read or written, node arrays gathered, atomics counted as
// read + write), independent of caching.
double alg_bytes(int which, int D, double np, double nn, double tb) {
  const double ns = (D * D) * (D * D + 1) / 2.0;
  switch (which) {
    case OSMPM_K_CG_PRODUCT:  // x, Atil per particle; z, p_prev, p_cur, Hp (rmw) per DOF, mass per node
      return np * (8.0 * D + tb * ns) + nn * (tb * 5.0 * D + 8.0);
    case OSMPM_K_CG_UPDATE:  // Hp (read, clear), p, r (rmw), z, del (rmw), diag per DOF + mask; mass per node
      return nn * (D * (tb * 8.0 + 1.0) + 8.0);
    case OSMPM_K_P2G:  // x, mass, flags; v, B per particle; mass and momentum (rmw) per node
      return np * (8.0 * (D + 1.0) + tb * (D + D * D) + 1.0) + nn * 16.0 * (1.0 + D);
    case OSMPM_K_G2P:  // x read and written, F read; v, B, F written; u and mass gathered per node
      return np * (16.0 * D + tb * (D + 3.0 * D * D)) + nn * 8.0 * (D + 1.0);
    case OSMPM_K_GRAD_HESS:  // x, vol, mat, F read; Atil written; u read, gradient rmw, diagonal rmw
      return np * (8.0 * (D + 1.0) + 4.0 + tb * (D * D + ns)) + nn * (8.0 * 3.0 * D + tb * 2.0 * D);
    default:
      return 0.0;
  }
}

// Copies the device error word and up to three partial arrays to pinned host
// memory, waits, and returns their host sums (fixed order).
struct Fetch {
  const double *p[3] = {nullptr, nullptr, nullptr};
  int n[3] = {0, 0, 0};
  double sum[3] = {0, 0, 0};
};

osmpm_status fetch(osmpm_ctx *c, Fetch &f, int *err_out) {
  size_t total = 1;
  for (int k = 0; k < 3; ++k) total += f.n[k];
  osmpm_status s = ensure_pin(c, total);
  if (s) return s;
  size_t off = 1;
  HIP_TRY(c, hipMemcpyAsync(c->h_pin, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  for (int k = 0; k < 3; ++k) {
    if (f.n[k] > 0)
      HIP_TRY(c, hipMemcpyAsync(c->h_pin + off, f.p[k], f.n[k] * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    off += f.n[k];
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  prof_harvest(c);
  int err = 0;
  std::memcpy(&err, c->h_pin, sizeof(int));
  off = 1;
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int i = 0; i < f.n[k]; ++i) acc += c->h_pin[off + i];
    f.sum[k] = acc;
    off += f.n[k];
  }
  *err_out = err;
  return OSMPM_OK;
}

osmpm_status device_error(osmpm_ctx *c, int err) {
  if (err & kErrOutOfGrid) return fail(c, OSMPM_E_OUT_OF_GRID, "a particle or node left its grid");
  if (err & kErrInverted) return fail(c, OSMPM_E_INVERTED, "det F <= 0 at an evaluated iterate");
  if (err & kErrTile) return fail(c, OSMPM_E_STATE, "particle binning inconsistent with positions");
  return OSMPM_OK;
}

osmpm_status check_launch(osmpm_ctx *c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, OSMPM_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return OSMPM_OK;
}

void zero_d(osmpm_ctx *c, double *a, int64_t n) {
  if (n > 0) k_fill<double><<<blocks_for(n), kBlock, 0, c->stream>>>(n, 0.0, a);
}
template <typename TB>
void zero_tb(osmpm_ctx *c, void *a, int64_t n) {
  if (n > 0) k_fill<TB><<<blocks_for(n), kBlock, 0, c->stream>>>(n, TB(0), static_cast<TB *>(a));
}
void zero_i64(osmpm_ctx *c, long long *a, int64_t n) {
  if (n > 0) k_fill_i64<<<blocks_for(n), kBlock, 0, c->stream>>>(n, a);
}
void zero_i32(osmpm_ctx *c, int *a, int64_t n) {
  if (n > 0) k_fill_i32<<<blocks_for(n), kBlock, 0, c->stream>>>(n, 0, a);
}

int ndof(const osmpm_domain *d) { return d->g.nn * d->D; }

size_t lds_p2g(const osmpm_domain *d) {
  return d->tg.nreg * (sizeof(long long) * (1 + kMaxGroups) + sizeof(double) * (1 + d->D));
}
size_t lds_grad(const osmpm_domain *d) { return d->tg.nreg * sizeof(double) * 3 * d->D; }
size_t lds_hvp(const osmpm_domain *d) { return d->tg.nreg * (sizeof(double) + d->tb) * d->D; }

double fixed_scale(const osmpm_domain *d) { return 4294967296.0 / d->m_ref; }
long long tau_fixed(const osmpm_domain *d) { return llrint(d->tau * fixed_scale(d)); }

// ---------------------------------------------------------------- sort + P2G
template <int D, typename TB>
osmpm_status sort_particles(osmpm_domain *d) {
  osmpm_ctx *c = d->ctx;
  const int n = d->np;
  PartBuf &a = d->pb[d->cur], &b = d->pb[d->cur ^ 1];
  zero_i32(c, d->count, d->nk);
  if (n > 0) {
    k_keys<D><<<blocks_for(n, 1 << 20), kBlock, 0, c->stream>>>(n, a.x, d->cap, d->g, d->tg, d->key, d->count, c->d_err);
  }
  k_scan<<<1, 1024, 0, c->stream>>>(d->nk, d->count, d->cell_start, d->cursor);
  if (n == 0) return check_launch(c);
  k_scatter<<<blocks_for(n, 1 << 20), kBlock, 0, c->stream>>>(n, d->key, d->cursor, d->perm);
  k_cellsort<<<blocks_for(d->nk, 1 << 20), kBlock, 0, c->stream>>>(d->nk, d->cell_start, d->perm);
  const int gb = blocks_for((int64_t)n * D * D, 2048);
  k_gather<double><<<gb, kBlock, 0, c->stream>>>(n, D, d->perm, a.x, b.x, d->cap);
  k_gather<TB><<<gb, kBlock, 0, c->stream>>>(n, D, d->perm, (const TB *)a.v, (TB *)b.v, d->cap);
  k_gather<TB><<<gb, kBlock, 0, c->stream>>>(n, D * D, d->perm, (const TB *)a.B, (TB *)b.B, d->cap);
  k_gather<TB><<<gb, kBlock, 0, c->stream>>>(n, D * D, d->perm, (const TB *)a.F, (TB *)b.F, d->cap);
  k_gather<double><<<gb, kBlock, 0, c->stream>>>(n, 1, d->perm, a.mass, b.mass, d->cap);
  k_gather<double><<<gb, kBlock, 0, c->stream>>>(n, 1, d->perm, a.vol, b.vol, d->cap);
  k_gather<int><<<gb, kBlock, 0, c->stream>>>(n, 1, d->perm, a.mat, b.mat, d->cap);
  k_gather<int><<<gb, kBlock, 0, c->stream>>>(n, 1, d->perm, a.id, b.id, d->cap);
  k_gather<uint8_t><<<gb, kBlock, 0, c->stream>>>(n, 1, d->perm, a.flags, b.flags, d->cap);
  d->cur ^= 1;
  return check_launch(c);
}

template <int D, typename TB>
osmpm_status p2g_impl(osmpm_domain *d, bool want_qall) {
  osmpm_ctx *c = d->ctx;
  osmpm_status s = sort_particles<D, TB>(d);
  if (s) return s;
  const int nn = d->g.nn;
  zero_d(c, d->m, nn);
  zero_d(c, d->vn, (int64_t)nn * D);
  const int want_q = (want_qall || d->bc.n_groups > 0) ? 1 : 0;
  if (want_q) {
    zero_i64(c, d->q_all, nn);
    zero_i64(c, d->qg, (int64_t)nn * std::max(d->bc.n_groups, 1));
  }
  const PartBuf &a = d->pb[d->cur];
  if (d->np > 0) {
    const double Dinv = 4.0 * d->g.inv_dx * d->g.inv_dx;
    launch(c, OSMPM_K_P2G, alg_bytes(OSMPM_K_P2G, D, d->np, nn, d->tb), -1, k_p2g<D, TB>, dim3(d->tg.nblocks),
           dim3(kBlock), (uint32_t)lds_p2g(d), d->tg, d->g, (const int *)d->cell_start, (const double *)a.x,
           (const TB *)a.v, (const TB *)a.B, (const double *)a.mass, (const uint8_t *)a.flags, d->cap, d->bc.n_groups,
           fixed_scale(d), Dinv, want_q, d->m, d->vn, d->q_all, d->qg, c->d_err);
  }
  k_p2g_final<D><<<blocks_for(nn, 1 << 20), kBlock, 0, c->stream>>>(d->g, d->m, d->vn, d->qg, d->bc, tau_fixed(d),
                                                                     d->bcg);
  d->have_p2g = true;
  return check_launch(c);
}

template <int D, typename TB>
osmpm_status g2p_impl(osmpm_domain *d, double dt) {
  osmpm_ctx *c = d->ctx;
  if (!d->have_p2g) return fail(c, OSMPM_E_STATE, "g2p before p2g");
  if (d->np == 0) return OSMPM_OK;
  PartBuf &a = d->pb[d->cur];
  launch(c, OSMPM_K_G2P, alg_bytes(OSMPM_K_G2P, D, d->np, d->g.nn, d->tb), -1, k_g2p<D, TB>,
         dim3(blocks_for(d->np, 1 << 20)), dim3(kBlock), 0, d->np, d->g, (const double *)d->m, (const double *)d->u, dt,
         a.x, (TB *)a.v, (TB *)a.B, (TB *)a.F, d->cap, c->d_err);
  return check_launch(c);
}

// ---------------------------------------------------------------- implicit solve
template <int D, typename TB>
osmpm_status solve_impl(osmpm_domain *d, double dt, int use_schwarz, const osmpm_solve_opts *o,
                        osmpm_solve_stats *st) {
  osmpm_ctx *c = d->ctx;
  if (!d->have_p2g) return fail(c, OSMPM_E_STATE, "solve before p2g");
  if (!(dt > 0.0)) return fail(c, OSMPM_E_INVALID_ARG, "dt must be positive");
  osmpm_solve_stats S{};
  const int nn = d->g.nn, nd = ndof(d);
  const PartBuf &a = d->pb[d->cur];
  k_bc_init<D><<<d->nb_node, kBlock, 0, c->stream>>>(d->g, d->m, d->vn, d->bcg, d->recv, d->vbc, use_schwarz, d->bc,
                                                     dt, d->fr, d->u, d->part_a);
  int err = 0;
  Fetch fm;
  fm.p[0] = d->part_a;
  fm.n[0] = d->nb_node;
  osmpm_status s = fetch(c, fm, &err);
  if (s) return s;
  const double gscale = fm.sum[0] * d->g.dx / (dt * dt);
  const size_t lg = lds_grad(d), lh = lds_hvp(d);
  for (int it = 0;; ++it) {
    zero_d(c, d->gg, nd);
    zero_tb<TB>(c, d->gd, nd);
    if (d->np > 0)
      launch(c, OSMPM_K_GRAD_HESS, alg_bytes(OSMPM_K_GRAD_HESS, D, d->np, nn, d->tb), -1, k_grad_hess<D, TB>,
             dim3(d->tg.nblocks), dim3(kBlock), (uint32_t)lg, d->tg, d->g, (const int *)d->cell_start,
             (const double *)a.x, (const TB *)a.F, (const double *)a.vol, (const int *)a.mat,
             (const double *)d->mu, (const double *)d->lam, d->cap, (const double *)d->u, 1, o->project_psd, d->gg,
             (TB *)d->gd, (TB *)d->Atil, c->d_err);
    k_grad_node<D, TB><<<d->nb_node, kBlock, 0, c->stream>>>(d->g, d->m, d->vn, d->u, d->fr, dt, o->gravity[0],
                                                             o->gravity[1], o->gravity[2], d->gg, (TB *)d->gd, 1,
                                                             d->part_a);
    Fetch fg;
    fg.p[0] = d->part_a;
    fg.n[0] = d->nb_node;
    if ((s = fetch(c, fg, &err))) return s;
    if ((s = device_error(c, err))) return s;
    const double gn = std::sqrt(fg.sum[0]);
    if (it == 0) S.gnorm0 = gn;
    S.gnorm = gn;
    const double tol = std::max(o->newton_rtol * S.gnorm0, o->newton_atol * gscale);
    if (gn <= tol) {
      S.converged = 1;
      break;
    }
    if (it == o->max_newton) break;
    // PCG on H del = -g
    k_cg_init<D, TB><<<d->nb_node, kBlock, 0, c->stream>>>(nd, d->gg, (const TB *)d->gd, d->fr, (TB *)d->r,
                                                           (TB *)d->z, (TB *)d->p0, (TB *)d->p1, (TB *)d->del,
                                                           (TB *)d->Hp, d->part_rz, d->part_rr, d->cg);
    // Batches of iterations between host checks: the first batch is sized
    // from the previous solve's count so the loop usually ends after one or
    // two checks; iterations launched after convergence exit at once.
    int launched = 0;
    int batch = std::max(4, std::min(d->cg_hint, o->max_cg));
    for (;;) {
      const int nb = std::min(batch, o->max_cg + 1 - launched);
      for (int j = 0; j < nb; ++j) {
        launch(c, OSMPM_K_CG_PRODUCT, alg_bytes(OSMPM_K_CG_PRODUCT, D, d->np, nn, d->tb), launched + j,
               k_cg_hvp<D, TB>, dim3(d->tg.nblocks), dim3(kBlock), (uint32_t)lh, d->tg, d->g,
               (const int *)d->cell_start, (const double *)a.x, (const TB *)d->Atil, d->cap, (const double *)d->m, dt,
               nd, (const TB *)d->z, (TB *)d->p0, (TB *)d->p1, (TB *)d->Hp, (const double *)d->part_rz,
               (const double *)d->part_rr, d->nb_node, o->cg_rtol, o->max_cg, d->part_q, d->cg);
        launch(c, OSMPM_K_CG_UPDATE, alg_bytes(OSMPM_K_CG_UPDATE, D, d->np, nn, d->tb), launched + j,
               k_cg_update<D, TB>, dim3(d->nb_node), dim3(kBlock), 0, nd, (const double *)d->m, dt,
               (const uint8_t *)d->fr, (const TB *)d->gd, (const TB *)d->p0, (const TB *)d->p1, (TB *)d->Hp,
               (TB *)d->r, (TB *)d->z, (TB *)d->del, (const double *)d->part_q, d->tg.nblocks, d->part_rz,
               d->part_rr, d->cg);
      }
      launched += nb;
      if ((s = check_launch(c))) return s;
      HIP_TRY(c, hipMemcpyAsync(c->h_pin, d->cg, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      CgState hs;
      std::memcpy(&hs, c->h_pin, sizeof(CgState));
      prof_harvest(c, hs.iter);
      if (hs.done || launched > o->max_cg) {
        S.cg_iters += hs.iter;
        d->cg_hint = hs.iter + 1;
        break;
      }
      batch = 4;
    }
    // halving line search on the exact energy difference
    double alpha = 1.0;
    bool accepted = false;
    for (int ls = 0; ls <= o->max_ls; ++ls) {
      if (d->np > 0)
        k_delta_energy_p<D, TB><<<d->nb_part, kBlock, 0, c->stream>>>(d->np, d->g, a.x, (const TB *)a.F, a.vol,
                                                                      a.mat, d->mu, d->lam, d->cap, d->u,
                                                                      (const TB *)d->del, alpha, d->part_b);
      k_delta_energy_n<D, TB><<<d->nb_node, kBlock, 0, c->stream>>>(d->g, d->m, d->vn, d->u, (const TB *)d->del, dt,
                                                                    alpha,
                                                                o->gravity[0], o->gravity[1], o->gravity[2],
                                                                d->part_a);
      Fetch fe;
      fe.p[0] = d->part_a;
      fe.n[0] = d->nb_node;
      fe.p[1] = d->part_b;
      fe.n[1] = d->np > 0 ? d->nb_part : 0;
      if ((s = fetch(c, fe, &err))) return s;
      const double dE = fe.sum[0] + fe.sum[1];
      if (dE < 0.0) {
        accepted = true;
        break;
      }
      if (ls == o->max_ls) break;
      alpha *= 0.5;
      S.ls_halvings += 1;
    }
    if (!accepted) {
      S.ls_failed = 1;
      break;
    }
    k_axpy<TB><<<blocks_for(nd), kBlock, 0, c->stream>>>(nd, alpha, (const TB *)d->del, d->u);
    S.newton_iters += 1;
  }
  if ((s = check_launch(c))) return s;
  if (st) *st = S;
  return OSMPM_OK;
}

// ---------------------------------------------------------------- interface
template <int D>
osmpm_status boundary_set(osmpm_domain *d) {
  osmpm_ctx *c = d->ctx;
  zero_i64(c, d->q_bnd, d->g.nn);
  const PartBuf &a = d->pb[d->cur];
  if (d->np > 0)
    k_qbnd<D><<<blocks_for(d->np, 1 << 20), kBlock, 0, c->stream>>>(d->np, d->g, a.x, a.mass, a.flags, d->cap,
                                                                     fixed_scale(d), d->q_bnd);
  k_gamma<<<blocks_for(d->g.nn, 1 << 20), kBlock, 0, c->stream>>>(d->g.nn, d->q_bnd, d->m, tau_fixed(d), d->gamma,
                                                                   d->recv);
  return check_launch(c);
}

template <int D>
osmpm_status interface_impl(osmpm_domain *B, osmpm_domain *S) {
  osmpm_ctx *c = B->ctx;
  osmpm_status s;
  if ((s = boundary_set<D>(B)) || (s = boundary_set<D>(S))) return s;
  zero_i32(c, c->d_count, 1);
  k_arbitrate<D><<<blocks_for(B->g.nn, 1 << 20), kBlock, 0, c->stream>>>(B->g, S->g, B->gamma, S->gamma, B->q_all,
                                                                          S->q_all, B->recv, S->recv, c->d_count);
  return check_launch(c);
}

template <int D>
osmpm_status project_impl(osmpm_domain *S, osmpm_domain *B, double eps_tol, const double *vS, double *out) {
  osmpm_ctx *c = B->ctx;
  zero_d(c, B->pnum, (int64_t)B->g.nn * D);
  zero_d(c, B->pden, B->g.nn);
  k_project_scatter<D><<<blocks_for(S->g.nn, 1 << 20), kBlock, 0, c->stream>>>(S->g, B->g, S->m, vS ? vS : S->vn,
                                                                                 B->pnum, B->pden, c->d_err);
  k_project_final<D><<<blocks_for(B->g.nn, 1 << 20), kBlock, 0, c->stream>>>(B->g.nn, B->recv, B->pnum, B->pden,
                                                                              eps_tol, out);
  return check_launch(c);
}

template <int D>
osmpm_status interp_impl(osmpm_domain *B, const double *vB, osmpm_domain *S, double *out) {
  osmpm_ctx *c = B->ctx;
  k_interp<D><<<blocks_for(S->g.nn, 1 << 20), kBlock, 0, c->stream>>>(B->g, S->g, B->m, vB ? vB : B->vn, S->recv,
                                                                       out, c->d_err);
  return check_launch(c);
}

osmpm_status copy_state(osmpm_domain *d, const PartBuf &from, PartBuf &to) {
  osmpm_ctx *c = d->ctx;
  const int D = d->D;
  const size_t cap = (size_t)d->cap;
  HIP_TRY(c, hipMemcpyAsync(to.x, from.x, cap * D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(to.v, from.v, cap * D * d->tb, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(to.B, from.B, cap * D * D * d->tb, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(to.F, from.F, cap * D * D * d->tb, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(to.mass, from.mass, cap * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(to.vol, from.vol, cap * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(to.mat, from.mat, cap * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(to.id, from.id, cap * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(to.flags, from.flags, cap * sizeof(uint8_t), hipMemcpyDeviceToDevice, c->stream));
  return OSMPM_OK;
}

template <int D>
osmpm_status residual(osmpm_domain *d, const double *a, const double *b, double *r_out) {
  osmpm_ctx *c = d->ctx;
  const int nb = blocks_for(d->g.nn);
  k_resid<D><<<nb, kBlock, 0, c->stream>>>(d->g.nn, d->recv, a, b, d->part_b);
  osmpm_status s = check_launch(c);
  if (s) return s;
  s = ensure_pin(c, 2 * nb + 1);
  if (s) return s;
  HIP_TRY(c, hipMemcpyAsync(c->h_pin, d->part_b, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double s1 = 0.0, s2 = 0.0;
  for (int i = 0; i < nb; ++i) {
    s1 += c->h_pin[2 * i];
    s2 += c->h_pin[2 * i + 1];
  }
  *r_out = std::sqrt(s1) / std::max(std::sqrt(s2), 1e-30);
  return OSMPM_OK;
}

void add_stats(int &nt, int &cg, int &ls, const osmpm_solve_stats &s) {
  nt += s.newton_iters;
  cg += s.cg_iters;
  ls += s.ls_halvings;
}

// One global frame of Alg. 1.  Buffers: B->w0 = Pi data of the current
// iteration, B->w1 = Pi data of the next, B->w2 = v_B^(k+1); S->w0 = I(v_B^n),
// S->w1 = I(v_B^(k+1)), S->w2 = previous I data for r_S.
template <int D, typename TB>
osmpm_status schwarz_impl(osmpm_domain *B, osmpm_domain *S, double dT, const osmpm_schwarz_opts *o,
                          osmpm_schwarz_stats *out) {
  osmpm_ctx *c = B->ctx;
  osmpm_schwarz_stats st{};
  osmpm_status s;
  const int M = o->M;
  const double dt = dT / (double)M;
  const int nB = B->g.nn * D, nS = S->g.nn * D;
  // Step 0
  if ((s = copy_state(S, S->pb[S->cur], S->st))) return s;
  if ((s = p2g_impl<D, TB>(B, true)) || (s = p2g_impl<D, TB>(S, true))) return s;
  if ((s = interface_impl<D>(B, S))) return s;
  if ((s = project_impl<D>(S, B, o->eps_tol, nullptr, B->w0))) return s;
  if ((s = interp_impl<D>(B, nullptr, S, S->w2))) return s;
  for (int k = 0; k < o->k_max; ++k) {
    osmpm_solve_stats ss{};
    // 1. coarse solve with Pi data
    HIP_TRY(c, hipMemcpyAsync(B->vbc, B->w0, nB * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if ((s = solve_impl<D, TB>(B, dT, 1, &o->coarse, &ss))) return s;
    add_stats(st.newton_B, st.cg_B, st.ls_B, ss);
    k_vel_from_u<D><<<blocks_for(B->g.nn, 1 << 20), kBlock, 0, c->stream>>>(B->g.nn, B->m, B->u, dT, B->w2);
    // 2. fine sub-cycling from the restored state
    if ((s = copy_state(S, S->st, S->pb[S->cur]))) return s;
    if ((s = p2g_impl<D, TB>(S, false))) return s;
    if ((s = interp_impl<D>(B, nullptr, S, S->w0))) return s;
    if ((s = interp_impl<D>(B, B->w2, S, S->w1))) return s;
    for (int m = 1; m <= M; ++m) {
      k_temporal<<<blocks_for(nS), kBlock, 0, c->stream>>>(nS, (double)m / (double)M, S->w0, S->w1, S->vbc);
      if ((s = solve_impl<D, TB>(S, dt, 1, &o->fine, &ss))) return s;
      add_stats(st.newton_S, st.cg_S, st.ls_S, ss);
      if ((s = g2p_impl<D, TB>(S, dt))) return s;
      if ((s = p2g_impl<D, TB>(S, false))) return s;
    }
    // 3. residuals
    if ((s = project_impl<D>(S, B, o->eps_tol, nullptr, B->w1))) return s;
    if ((s = residual<D>(B, B->w1, B->w0, &st.r_B))) return s;
    if ((s = residual<D>(S, S->w1, S->w2, &st.r_S))) return s;
    std::swap(B->w0, B->w1);
    std::swap(S->w2, S->w1);
    st.iters = k + 1;
    if (st.r_B <= o->eps_conv && st.r_S <= o->eps_conv) {
      st.converged = 1;
      break;
    }
  }
  // 4. coarse G2P + advection with the last coarse solution
  if ((s = g2p_impl<D, TB>(B, dT))) return s;
  // receiver counts and ambiguous pairs
  {
    const int nbB = B->g.nn, nbS = S->g.nn;
    std::vector<uint8_t> hb(nbB), hs(nbS);
    HIP_TRY(c, hipMemcpyAsync(hb.data(), B->recv, nbB, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(hs.data(), S->recv, nbS, hipMemcpyDeviceToHost, c->stream));
    int amb = 0;
    HIP_TRY(c, hipMemcpyAsync(&amb, c->d_count, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (uint8_t v : hb) st.n_recv_B += v;
    for (uint8_t v : hs) st.n_recv_S += v;
    st.n_amb = amb;
  }
  int err = 0;
  Fetch f0;
  if ((s = fetch(c, f0, &err))) return s;
  if ((s = device_error(c, err))) return s;
  if (out) *out = st;
  return OSMPM_OK;
}

// Tile geometry of a domain for tile shape T.
TileGeom make_tiles(const osmpm_grid &gd, const int *T) {
  TileGeom tg{};
  tg.nreg = 1;
  tg.tvol = 1;
  tg.ntiles = 1;
  for (int a = 0; a < 3; ++a) {
    if (a < gd.dim) {
      tg.T[a] = T[a];
      tg.nt[a] = (gd.n_nodes[a] - 2 + T[a] - 1) / T[a];
      tg.R[a] = T[a] + 2;
    } else {
      tg.T[a] = 1;
      tg.nt[a] = 1;
      tg.R[a] = 1;
    }
    tg.nreg *= tg.R[a];
    tg.tvol *= tg.T[a];
    tg.ntiles *= tg.nt[a];
  }
  tg.nblocks = ((tg.ntiles + 7) / 8) * 8;
  return tg;
}

}  // namespace

// ====================================================================== ABI
#define DISPATCH(dim, call) ((dim) == 2 ? call<2> : call<3>)
// Dispatch on dimension and bulk type of a domain.
#define DISPATCH2(dom, call)                                                                              \
  ((dom)->D == 2 ? ((dom)->precision == OSMPM_MIXED ? call<2, float> : call<2, double>)                 \
                 : ((dom)->precision == OSMPM_MIXED ? call<3, float> : call<3, double>))

extern "C" {

osmpm_status osmpm_ctx_create(int32_t device, void *stream, osmpm_ctx **out) {
  if (!out) return OSMPM_E_INVALID_ARG;
  *out = nullptr;
  auto *c = new osmpm_ctx();
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return OSMPM_E_DEVICE;
  }
  c->stream = (hipStream_t)stream;
  if (hipMalloc(&c->d_err, sizeof(int)) != hipSuccess || hipMalloc(&c->d_count, sizeof(int)) != hipSuccess) {
    delete c;
    return OSMPM_E_NO_MEMORY;
  }
  (void)hipMemsetAsync(c->d_err, 0, sizeof(int), c->stream);
  (void)hipMemsetAsync(c->d_count, 0, sizeof(int), c->stream);
  if (ensure_pin(c, 1 << 16)) {
    delete c;
    return OSMPM_E_NO_MEMORY;
  }
  (void)hipStreamSynchronize(c->stream);
  *out = c;
  return OSMPM_OK;
}

osmpm_status osmpm_ctx_set_stream(osmpm_ctx *ctx, void *stream) {
  if (!ctx) return OSMPM_E_INVALID_ARG;
  ctx->stream = (hipStream_t)stream;
  return OSMPM_OK;
}

osmpm_status osmpm_sync(osmpm_ctx *ctx) {
  if (!ctx) return OSMPM_E_INVALID_ARG;
  int err = 0;
  Fetch f;
  osmpm_status s = fetch(ctx, f, &err);
  if (s) return s;
  return device_error(ctx, err);
}

osmpm_status osmpm_profile_enable(osmpm_ctx *ctx, int32_t enable) {
  if (!ctx) return OSMPM_E_INVALID_ARG;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  prof_harvest(ctx);
  for (auto &sl : ctx->slots) sl = ProfSlot{};
  ctx->prof = enable != 0;
  return OSMPM_OK;
}

osmpm_status osmpm_profile_query(osmpm_ctx *ctx, int32_t which, int64_t *launches, double *total_ms,
                                 double *bytes) {
  if (!ctx || which < 0 || which >= OSMPM_K_COUNT) return OSMPM_E_INVALID_ARG;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  prof_harvest(ctx);
  if (launches) *launches = ctx->slots[which].launches;
  if (total_ms) *total_ms = ctx->slots[which].ms;
  if (bytes) *bytes = ctx->slots[which].bytes;
  return OSMPM_OK;
}

const char *osmpm_last_error(const osmpm_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

void osmpm_ctx_destroy(osmpm_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(ctx->d_err);
  (void)hipFree(ctx->d_count);
  if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
  prof_harvest(ctx);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
}

osmpm_status osmpm_domain_create(osmpm_ctx *ctx, const osmpm_grid *grid, int32_t precision, int64_t capacity,
                                 const int32_t *tile_host, osmpm_domain **out) {
  if (!ctx || !grid || !out) return OSMPM_E_INVALID_ARG;
  *out = nullptr;
  if (grid->dim != 2 && grid->dim != 3) return fail(ctx, OSMPM_E_INVALID_ARG, "dim must be 2 or 3");
  if (precision != OSMPM_FP64 && precision != OSMPM_MIXED) return fail(ctx, OSMPM_E_INVALID_ARG, "bad precision");
  for (int a = 0; a < grid->dim; ++a)
    if (grid->n_nodes[a] < 3) return fail(ctx, OSMPM_E_INVALID_ARG, "grid needs >= 3 nodes per axis");
  if (grid->dim == 2 && grid->n_nodes[2] != 1) return fail(ctx, OSMPM_E_INVALID_ARG, "n_nodes[2] must be 1 in 2D");
  if (!(grid->h0 > 0.0) || grid->dx_q <= 0 || capacity < 0 || capacity > (1LL << 30))
    return fail(ctx, OSMPM_E_INVALID_ARG, "bad grid spacing or capacity");
  int T[3] = {grid->dim == 2 ? 8 : 4, grid->dim == 2 ? 8 : 4, grid->dim == 2 ? 1 : 4};
  if (tile_host)
    for (int a = 0; a < grid->dim; ++a)
      if (tile_host[a] > 0) T[a] = tile_host[a];
  auto *d = new osmpm_domain();
  d->ctx = ctx;
  d->D = grid->dim;
  d->desc = *grid;
  d->precision = precision;
  d->tb = (precision == OSMPM_MIXED) ? sizeof(float) : sizeof(double);
  d->cap = std::max<int64_t>(capacity, 1);
  GridDev &g = d->g;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = (a < grid->dim) ? grid->n_nodes[a] : 1;
    g.origin_q[a] = (a < grid->dim) ? grid->origin_q[a] : 0;
    g.origin[a] = (double)g.origin_q[a] * grid->h0;
  }
  g.nn = g.n[0] * g.n[1] * g.n[2];
  g.h0 = grid->h0;
  g.dx_q = grid->dx_q;
  g.dx = (double)grid->dx_q * grid->h0;
  g.inv_dx = 1.0 / g.dx;
  d->tg = make_tiles(*grid, T);
  if ((size_t)d->tg.nreg * sizeof(double) * (2 + d->D + kMaxGroups) > 60 * 1024) {
    delete d;
    return fail(ctx, OSMPM_E_INVALID_ARG, "tile too large for LDS");
  }
  d->nk = d->tg.ntiles * d->tg.tvol;
  const int D = d->D, nn = g.nn, nd = nn * D;
  const size_t cap = (size_t)d->cap;
  d->nb_node = blocks_for(nd);
  d->nb_part = blocks_for(d->cap);
  osmpm_status s = OSMPM_OK;
  auto part_alloc = [&](PartBuf &p) {
    if (!s) s = dalloc(d, &p.x, cap * D);
    if (!s) s = dalloc_bytes(d, &p.v, cap * D * d->tb);
    if (!s) s = dalloc_bytes(d, &p.B, cap * D * D * d->tb);
    if (!s) s = dalloc_bytes(d, &p.F, cap * D * D * d->tb);
    if (!s) s = dalloc(d, &p.mass, cap);
    if (!s) s = dalloc(d, &p.vol, cap);
    if (!s) s = dalloc(d, &p.mat, cap);
    if (!s) s = dalloc(d, &p.id, cap);
    if (!s) s = dalloc(d, &p.flags, cap);
  };
  part_alloc(d->pb[0]);
  part_alloc(d->pb[1]);
  part_alloc(d->st);
  const int ns = (D * D) * (D * D + 1) / 2;
  const int nbmax = std::max({d->nb_node, d->nb_part, d->tg.nblocks, blocks_for(nn)}) * 2 + 8;
  if (!s) s = dalloc(d, &d->key, cap);
  if (!s) s = dalloc(d, &d->perm, cap);
  if (!s) s = dalloc(d, &d->count, (size_t)d->nk + 1);
  if (!s) s = dalloc(d, &d->cell_start, (size_t)d->nk + 1);
  if (!s) s = dalloc(d, &d->cursor, (size_t)d->nk + 1);
  if (!s) s = dalloc(d, &d->m, nn);
  if (!s) s = dalloc(d, &d->vn, nd);
  if (!s) s = dalloc(d, &d->u, nd);
  if (!s) s = dalloc(d, &d->vbc, nd);
  if (!s) s = dalloc(d, &d->bcg, nd);
  if (!s) s = dalloc(d, &d->gamma, nn);
  if (!s) s = dalloc(d, &d->recv, nn);
  if (!s) s = dalloc(d, &d->fr, nd);
  if (!s) s = dalloc(d, &d->q_all, nn);
  if (!s) s = dalloc(d, &d->q_bnd, nn);
  if (!s) s = dalloc(d, &d->qg, (size_t)nn * kMaxGroups);
  if (!s) s = dalloc(d, &d->gg, nd);
  if (!s) s = dalloc_bytes(d, &d->gd, nd * d->tb);
  if (!s) s = dalloc_bytes(d, &d->r, nd * d->tb);
  if (!s) s = dalloc_bytes(d, &d->z, nd * d->tb);
  if (!s) s = dalloc_bytes(d, &d->p0, nd * d->tb);
  if (!s) s = dalloc_bytes(d, &d->p1, nd * d->tb);
  if (!s) s = dalloc_bytes(d, &d->del, nd * d->tb);
  if (!s) s = dalloc_bytes(d, &d->Hp, nd * d->tb);
  if (!s) s = dalloc_bytes(d, &d->Atil, cap * ns * d->tb);
  if (!s) s = dalloc(d, &d->cg, 1);
  if (!s) s = dalloc(d, &d->part_a, nbmax);
  if (!s) s = dalloc(d, &d->part_b, nbmax);
  if (!s) s = dalloc(d, &d->part_q, nbmax);
  if (!s) s = dalloc(d, &d->part_rz, nbmax);
  if (!s) s = dalloc(d, &d->part_rr, nbmax);
  if (!s) s = dalloc(d, &d->pnum, nd);
  if (!s) s = dalloc(d, &d->pden, nn);
  if (!s) s = dalloc(d, &d->w0, nd);
  if (!s) s = dalloc(d, &d->w1, nd);
  if (!s) s = dalloc(d, &d->w2, nd);
  if (!s) s = dalloc(d, &d->w3, nd);
  if (!s) s = dalloc(d, &d->mu, 64);
  if (!s) s = dalloc(d, &d->lam, 64);
  if (s) {
    osmpm_domain_destroy(d);
    return s;
  }
  // defined initial contents
  zero_d(ctx, d->vbc, nd);
  zero_d(ctx, d->u, nd);
  zero_d(ctx, d->m, nn);
  (void)hipMemsetAsync(d->recv, 0, nn, ctx->stream);
  (void)hipMemsetAsync(d->gamma, 0, nn, ctx->stream);
  (void)hipMemsetAsync(d->q_all, 0, nn * sizeof(long long), ctx->stream);
  *out = d;
  return check_launch(ctx);
}

void osmpm_domain_destroy(osmpm_domain *dom) {
  if (!dom) return;
  if (dom->ctx) (void)hipStreamSynchronize(dom->ctx->stream);
  for (void *p : dom->allocs) (void)hipFree(p);
  delete dom;
}

osmpm_status osmpm_domain_set_materials(osmpm_domain *d, const osmpm_material *mats, int32_t n_mat) {
  if (!d || !mats || n_mat < 1 || n_mat > 64) return OSMPM_E_INVALID_ARG;
  std::vector<double> mu(n_mat), lam(n_mat);
  for (int i = 0; i < n_mat; ++i) {
    const double E = mats[i].E, nu = mats[i].nu;
    if (!(E >= 0.0) || !(nu > -1.0 && nu < 0.5)) return fail(d->ctx, OSMPM_E_INVALID_ARG, "bad material");
    mu[i] = E / (2.0 * (1.0 + nu));
    lam[i] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  }
  osmpm_ctx *c = d->ctx;
  HIP_TRY(c, hipMemcpyAsync(d->mu, mu.data(), n_mat * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d->lam, lam.data(), n_mat * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  d->n_mat = n_mat;
  return OSMPM_OK;
}

osmpm_status osmpm_domain_set_particles(osmpm_domain *d, int64_t n, const double *x, const double *v, const double *B,
                                        const double *F, const double *mass, const double *vol, const int32_t *mat,
                                        const uint8_t *flags) {
  if (!d || n < 0 || n > d->cap) return OSMPM_E_INVALID_ARG;
  if (n > 0 && (!x || !v || !B || !F || !mass || !vol || !mat || !flags)) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  const int D = d->D;
  PartBuf &p = d->pb[d->cur];
  d->np = (int)n;
  if (n > 0) {
    const int gb = blocks_for(n * D * D, 2048);
    k_aos_to_soa<double><<<gb, kBlock, 0, c->stream>>>(n, D, x, p.x, d->cap);
    if (d->precision == OSMPM_MIXED) {
      k_aos_to_soa<float><<<gb, kBlock, 0, c->stream>>>(n, D, v, (float *)p.v, d->cap);
      k_aos_to_soa<float><<<gb, kBlock, 0, c->stream>>>(n, D * D, B, (float *)p.B, d->cap);
      k_aos_to_soa<float><<<gb, kBlock, 0, c->stream>>>(n, D * D, F, (float *)p.F, d->cap);
    } else {
      k_aos_to_soa<double><<<gb, kBlock, 0, c->stream>>>(n, D, v, (double *)p.v, d->cap);
      k_aos_to_soa<double><<<gb, kBlock, 0, c->stream>>>(n, D * D, B, (double *)p.B, d->cap);
      k_aos_to_soa<double><<<gb, kBlock, 0, c->stream>>>(n, D * D, F, (double *)p.F, d->cap);
    }
    HIP_TRY(c, hipMemcpyAsync(p.mass, mass, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(p.vol, vol, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(p.mat, mat, n * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(p.flags, flags, n * sizeof(uint8_t), hipMemcpyDeviceToDevice, c->stream));
    k_iota<<<blocks_for(n), kBlock, 0, c->stream>>>((int)n, p.id);
  }
  d->have_p2g = false;
  return check_launch(c);
}

osmpm_status osmpm_domain_set_selection(osmpm_domain *d, double m_ref, double tau) {
  if (!d || !(m_ref > 0.0) || !(tau >= 0.0)) return OSMPM_E_INVALID_ARG;
  d->m_ref = m_ref;
  d->tau = tau;
  return OSMPM_OK;
}

osmpm_status osmpm_domain_set_scene_bc(osmpm_domain *d, int32_t n_groups, const int32_t *kind, const int32_t *mask,
                                       const double *params) {
  if (!d || n_groups < 0 || n_groups > kMaxGroups) return OSMPM_E_INVALID_ARG;
  if (n_groups > 0 && (!kind || !mask || !params)) return OSMPM_E_INVALID_ARG;
  SceneBC bc{};
  bc.n_groups = n_groups;
  for (int gi = 0; gi < n_groups; ++gi) {
    if (kind[gi] < 0 || kind[gi] > 2 || (kind[gi] == 2 && d->D != 3))
      return fail(d->ctx, OSMPM_E_INVALID_ARG, "bad scene BC kind");
    bc.kind[gi] = kind[gi];
    bc.mask[gi] = mask[gi];
    for (int k = 0; k < 8; ++k) bc.param[gi][k] = params[gi * 8 + k];
  }
  d->bc = bc;
  return OSMPM_OK;
}

osmpm_status osmpm_p2g(osmpm_domain *d) {
  if (!d) return OSMPM_E_INVALID_ARG;
  return DISPATCH2(d, p2g_impl)(d, true);
}

osmpm_status osmpm_implicit_solve(osmpm_domain *d, double dt, int32_t use_schwarz_bc, const osmpm_solve_opts *o,
                                  osmpm_solve_stats *st) {
  if (!d || !o) return OSMPM_E_INVALID_ARG;
  if (o->max_newton < 0 || o->max_cg < 0 || o->max_ls < 0) return OSMPM_E_INVALID_ARG;
  return DISPATCH2(d, solve_impl)(d, dt, use_schwarz_bc, o, st);
}

osmpm_status osmpm_g2p(osmpm_domain *d, double dt) {
  if (!d || !(dt > 0.0)) return OSMPM_E_INVALID_ARG;
  return DISPATCH2(d, g2p_impl)(d, dt);
}

static bool pair_ok(const osmpm_domain *B, const osmpm_domain *S) {
  return B && S && B->ctx == S->ctx && B->D == S->D && B->desc.h0 == S->desc.h0 && B->m_ref == S->m_ref &&
         B->precision == S->precision;
}

osmpm_status osmpm_interface_build(osmpm_domain *B, osmpm_domain *S, int32_t *n_amb) {
  if (!pair_ok(B, S)) return OSMPM_E_INVALID_ARG;
  if (!B->have_p2g || !S->have_p2g) return fail(B->ctx, OSMPM_E_STATE, "interface before p2g");
  osmpm_status s = DISPATCH(B->D, interface_impl)(B, S);
  if (s || !n_amb) return s;
  osmpm_ctx *c = B->ctx;
  int v = 0;
  HIP_TRY(c, hipMemcpyAsync(&v, c->d_count, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *n_amb = v;
  return OSMPM_OK;
}

osmpm_status osmpm_project_S_to_B(osmpm_domain *S, osmpm_domain *B, double eps_tol, const double *vS, double *out) {
  if (!pair_ok(B, S) || !out || !(eps_tol >= 0.0)) return OSMPM_E_INVALID_ARG;
  return DISPATCH(B->D, project_impl)(S, B, eps_tol, vS, out);
}

osmpm_status osmpm_interp_B_to_S(osmpm_domain *B, const double *vB, osmpm_domain *S, double *out) {
  if (!pair_ok(B, S) || !out) return OSMPM_E_INVALID_ARG;
  return DISPATCH(B->D, interp_impl)(B, vB, S, out);
}

osmpm_status osmpm_temporal_interp(osmpm_ctx *ctx, int64_t n, int32_t m, int32_t M, const double *vn,
                                   const double *vn1, double *out) {
  if (!ctx || n < 0 || M < 1 || m < 0 || m > M || (n > 0 && (!vn || !vn1 || !out))) return OSMPM_E_INVALID_ARG;
  if (n == 0) return OSMPM_OK;
  k_temporal<<<blocks_for(n), kBlock, 0, ctx->stream>>>(n, (double)m / (double)M, vn, vn1, out);
  return check_launch(ctx);
}

osmpm_status osmpm_set_schwarz_bc(osmpm_domain *d, const double *vbc) {
  if (!d || !vbc) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  HIP_TRY(c, hipMemcpyAsync(d->vbc, vbc, (size_t)ndof(d) * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return OSMPM_OK;
}

osmpm_status osmpm_schwarz_frame(osmpm_domain *B, osmpm_domain *S, double dT, const osmpm_schwarz_opts *o,
                                 osmpm_schwarz_stats *st) {
  if (!pair_ok(B, S) || !o || !(dT > 0.0) || o->M < 1 || o->k_max < 1 || !(o->eps_tol >= 0.0))
    return OSMPM_E_INVALID_ARG;
  return DISPATCH2(B, schwarz_impl)(B, S, dT, o, st);
}

osmpm_status osmpm_single_frame(osmpm_domain *d, double dt, const osmpm_solve_opts *o, osmpm_solve_stats *st) {
  if (!d || !o || !(dt > 0.0)) return OSMPM_E_INVALID_ARG;
  osmpm_status s = DISPATCH2(d, p2g_impl)(d, false);
  if (s) return s;
  if ((s = DISPATCH2(d, solve_impl)(d, dt, 0, o, st))) return s;
  if ((s = DISPATCH2(d, g2p_impl)(d, dt))) return s;
  return osmpm_sync(d->ctx);
}

osmpm_status osmpm_get_particles(osmpm_domain *d, double *x, double *v, double *B, double *F, int32_t *id) {
  if (!d) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  const int D = d->D;
  const int64_t n = d->np;
  if (n == 0) return OSMPM_OK;
  const PartBuf &p = d->pb[d->cur];
  const int gb = blocks_for(n * D * D, 2048);
  if (x) k_soa_to_aos<double><<<gb, kBlock, 0, c->stream>>>(n, D, p.x, d->cap, x);
  if (d->precision == OSMPM_MIXED) {
    if (v) k_soa_to_aos<float><<<gb, kBlock, 0, c->stream>>>(n, D, (const float *)p.v, d->cap, v);
    if (B) k_soa_to_aos<float><<<gb, kBlock, 0, c->stream>>>(n, D * D, (const float *)p.B, d->cap, B);
    if (F) k_soa_to_aos<float><<<gb, kBlock, 0, c->stream>>>(n, D * D, (const float *)p.F, d->cap, F);
  } else {
    if (v) k_soa_to_aos<double><<<gb, kBlock, 0, c->stream>>>(n, D, (const double *)p.v, d->cap, v);
    if (B) k_soa_to_aos<double><<<gb, kBlock, 0, c->stream>>>(n, D * D, (const double *)p.B, d->cap, B);
    if (F) k_soa_to_aos<double><<<gb, kBlock, 0, c->stream>>>(n, D * D, (const double *)p.F, d->cap, F);
  }
  if (id) HIP_TRY(c, hipMemcpyAsync(id, p.id, n * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
  return check_launch(c);
}

osmpm_status osmpm_get_grid(osmpm_domain *d, double *m, double *vn, double *u) {
  if (!d) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  const size_t nn = d->g.nn, nd = nn * d->D;
  if (m) HIP_TRY(c, hipMemcpyAsync(m, d->m, nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (vn) HIP_TRY(c, hipMemcpyAsync(vn, d->vn, nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (u) HIP_TRY(c, hipMemcpyAsync(u, d->u, nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return OSMPM_OK;
}

osmpm_status osmpm_get_sets(osmpm_domain *d, uint8_t *gamma, uint8_t *recv, int64_t *q_all) {
  if (!d) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  const size_t nn = d->g.nn;
  if (gamma) HIP_TRY(c, hipMemcpyAsync(gamma, d->gamma, nn, hipMemcpyDeviceToDevice, c->stream));
  if (recv) HIP_TRY(c, hipMemcpyAsync(recv, d->recv, nn, hipMemcpyDeviceToDevice, c->stream));
  if (q_all) HIP_TRY(c, hipMemcpyAsync(q_all, d->q_all, nn * sizeof(int64_t), hipMemcpyDeviceToDevice, c->stream));
  return OSMPM_OK;
}

osmpm_status osmpm_get_sort(osmpm_domain *d, int32_t *perm, int32_t *cell_start) {
  if (!d) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  if (perm && d->np > 0)
    HIP_TRY(c, hipMemcpyAsync(perm, d->perm, (size_t)d->np * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
  if (cell_start)
    HIP_TRY(c, hipMemcpyAsync(cell_start, d->cell_start, ((size_t)d->nk + 1) * sizeof(int), hipMemcpyDeviceToDevice,
                              c->stream));
  return OSMPM_OK;
}

osmpm_status osmpm_domain_info(osmpm_domain *d, int64_t *n_particles, int64_t *n_nodes, int64_t *n_keys) {
  if (!d) return OSMPM_E_INVALID_ARG;
  if (n_particles) *n_particles = d->np;
  if (n_nodes) *n_nodes = d->g.nn;
  if (n_keys) *n_keys = d->nk;
  return OSMPM_OK;
}

}  // extern "C"
