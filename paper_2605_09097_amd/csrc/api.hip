// Host side of the C ABI declared in include/osmpm.h: handle management and
// the sequencing of the binning / P2G / G2P pipelines, the implicit solve
// and the multiplicative Schwarz frame of Alg. 1.
//
// All work runs on groups of domains: a group holds n domains on one side
// (single-domain work) or n coarse/fine pairs on two sides (Schwarz work), and
// every stage is one launch over the whole group (blockIdx.y = domain).  A
// single domain is a group of one.  Newton, CG and line-search decisions are
// taken on the device per domain, so the host queues a fixed cycle of
// launches and reads one small status block per cycle: the solve states, the
// CG states, the Schwarz residual sums and the device error word.  All
// arithmetic on particles and nodes runs in the kernels of kernels.hip.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <hip/hip_ext.h>

#include "../../include/osmpm.h"
#include "kernels.hpp"

using namespace osmpm;

// Device work region of the entry point that allocates nothing (64 MiB per
// device; see fixed_region_setup).
constexpr size_t kFixedRegionBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kFixedRegionBytes];

namespace {

// Workgroups of a one-item-per-thread launch (at most kMaxBlocks; a domain's
// particle, node and bin counts are limited to kMaxItems so that such a
// launch covers all of them).
constexpr int kMaxBlocks = 1 << 20;
// Tile workgroups above which a solve sizes its tangent and CG launches to
// the working workgroups (one status read per solve).
constexpr int kSizedLaunch = 4096;
constexpr int64_t kMaxItems = (int64_t)kMaxBlocks * kBlock;

int blocks_for(int64_t n, int cap_blocks = kMaxBlocks) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap_blocks) b = cap_blocks;
  return (int)b;
}

int particle_blocks_host(int64_t np) { return blocks_for(np, 1024); }

// Kernel timing: start/stop timestamps of the dispatch of every instrumented
// launch while profiling is enabled.
struct ProfPending {
  hipEvent_t a, b;
  int which;
  double bytes;
  int cg_iter;  // index of a CG launch within its cycle, kCgSpan for a whole cycle's CG launches, -1 otherwise
};
constexpr int kCgSpan = -2;
struct ProfSlot {
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0;
};

// Explicit HIP graph under construction: launches append kernel nodes in a
// chain instead of being enqueued.
struct GraphBuild {
  hipGraph_t graph = nullptr;
  hipGraphNode_t last = nullptr;
  hipError_t err = hipSuccess;
};

// A cached solve cycle: key (launch count, step, solver options) and the
// instantiated graph.
struct CycleGraph {
  int b = 0;
  int grid_t = 0, grid_cg = 0;  // launch sizes of the tangent pass and the CG iteration
  double dt = 0.0;
  osmpm_solve_opts o{};
  hipGraphExec_t exec = nullptr;
};

// A cached whole Schwarz iteration of a two-sided group (fixed-schedule
// solves only): key (iteration class, frame step, Schwarz options) and the
// instantiated graph.  Iteration classes: 0 the first iteration (cold
// solves), 1 and 2 later iterations of odd and even index (the work-buffer
// roles alternate).
struct IterGraph {
  int cls = 0;
  double dT = 0.0;
  osmpm_schwarz_opts o{};
  hipGraphExec_t exec = nullptr;
};

// Work buffer indices understood by the kernels (see wbuf).
constexpr int kBufVn = 4, kBufVbc = 5;
// Partial-sum arrays per domain: two scalar reductions and the CG's three
// inner products at two parities.
constexpr int kPartArrays = 8;

}  // namespace

struct osmpm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char *h_pin = nullptr;  // pinned staging of status reads
  size_t h_pin_bytes = 0;
  std::string last_error;
  bool prof = false;
  ProfSlot slots[OSMPM_K_COUNT];
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfPending> pending;
  std::vector<osmpm_batch *> groups;  // every live group (error words)
  uint64_t next_uid = 1;
  int graphs = 0;                 // 1: replay solve cycles as HIP graphs; 2: also whole Schwarz iterations
  int cg_split = -1;              // CG scalars: 0 fused, 1 separate launch, -1 by size
  GraphBuild *rec = nullptr;      // graph being built (launches become nodes)
};

// Particle arrays, component-major [rows][capacity].  Positions, masses and
// volumes are FP64; velocities, affine matrices and deformation gradients
// are stored in the domain's bulk type (FP64, or FP32 in the mixed path).
struct osmpm_domain {
  osmpm_ctx *ctx = nullptr;
  uint64_t uid = 0;
  uint64_t version = 1;  // bumped when the device descriptor changes
  int D = 2;
  osmpm_grid desc{};
  GridDev g{};
  TileGeom tg{};
  int precision = 0;
  size_t tb = sizeof(double);  // bytes of the bulk type
  int64_t cap = 0;
  int np = 0;
  PartPtrs pb[2]{}, st{};
  int cur = 0;             // host mirror of *d_cur
  int *d_cur = nullptr;    // current particle buffer (device)
  int nk = 0;
  int *key = nullptr, *count = nullptr, *cell_start = nullptr, *cursor = nullptr, *perm = nullptr, *lperm = nullptr;
  int *tcount = nullptr;
  TileSlot *tl = nullptr;  // work lists (see DomDesc)
  int *nlist = nullptr, *ncnt = nullptr, *lcnt = nullptr;
  int n_mat = 0;
  double *mu = nullptr, *lam = nullptr;
  std::vector<double> E_h, nu_h;  // host copy of the material table
  double *tau_y = nullptr;        // von Mises yield stress per material (device)
  bool plastic = false;           // some material yields
  double m_ref = 1.0, tau = 0.0;
  SceneBC bc{};
  double *m = nullptr, *vn = nullptr, *u = nullptr, *vbc = nullptr, *gg = nullptr;
  int8_t *bcg = nullptr;
  uint8_t *gamma = nullptr, *recv = nullptr, *fr = nullptr;
  long long *q_all = nullptr, *q_bnd = nullptr, *qg = nullptr;
  void *gd = nullptr, *cr[2] = {}, *cs[2] = {}, *cw[3] = {}, *cu = nullptr, *cp = nullptr, *del = nullptr,
       *Atil = nullptr;
  double *pnum = nullptr, *pden = nullptr, *w0 = nullptr, *w1 = nullptr, *w2 = nullptr, *w3 = nullptr;
  int *flink = nullptr;    // fine-fine links [node][2] (multi groups)
  double *warm = nullptr;  // warm-start slots (see DomDesc), allocated on first use
  int warm_slots = 0;
  int cg_hint = 8;  // iterations of the last CG solve (sizes the next batch of launches)
  bool have_p2g = false;
  bool have_solve = false;  // an implicit solve since the last P2G (u is then zero on inactive nodes)
  // uid of the group whose status holds the live-tile and active-node counts
  // of the current work lists (the last group to bin this domain or rebuild
  // them; 0: none)
  uint64_t lists_by = 0;
  osmpm_batch *solo = nullptr;  // this domain as a group of one
  osmpm_batch *pair = nullptr;  // this coarse domain paired with a fine one
  uint64_t pair_uid = 0;
  std::vector<void *> allocs;
};

// Launch extents of one side of a group: maxima over its domains.
struct Ext {
  int max_np = 0, max_nn = 0, max_ndof = 0, max_nk = 0;
  int tile_blocks = 8, node_blocks = 1, part_blocks = 1, nn_blocks = 1;
  size_t lds_p2g = 0, lds_grad = 0, lds_hvp = 0;
};

namespace {
struct RunRecord;  // multi-frame run record of a Schwarz batch (defined with the reverse mode)
void run_free(RunRecord *r);
}  // namespace

// Status block read back once per cycle (one copy).
struct StatusHdr {
  int err;
  int pad[15];
};

struct osmpm_batch {
  bool multi = false;  // one coarse domain (repeated on side 0) and k fine domains
  osmpm_ctx *c = nullptr;
  uint64_t uid = 0;  // unique in the context (a freed group's address may be reused)
  int D = 2, precision = 0;
  size_t tb = sizeof(double);
  int n = 0, sides = 1;
  bool dead = false;
  std::vector<osmpm_domain *> dom[2];
  std::vector<uint64_t> stamp_uid[2], stamp_ver[2];
  std::vector<DomDesc> hdd[2];
  DomDesc *dd[2] = {nullptr, nullptr};
  int *active[2] = {nullptr, nullptr};
  std::vector<int> act[2];  // host mirror of active (-1: unknown)
  // status block: header, n_amb[n], n_recv[2][n], resid[2][n][2], SolveState[2][n], CgState[2][n]
  char *status = nullptr;
  char *h_status = nullptr;  // pinned host copy of the status block
  size_t status_bytes = 0;
  size_t off_amb = 0, off_recv = 0, off_res = 0, off_ss = 0, off_cg = 0;
  int *err = nullptr, *n_amb = nullptr, *n_recv = nullptr;
  double *res = nullptr;
  SolveState *ss[2] = {nullptr, nullptr};
  CgState *cg[2] = {nullptr, nullptr};
  double *parts = nullptr;
  int stride = 0;
  Ext ext[2];
  std::vector<double> bytes[2][OSMPM_K_COUNT];  // algorithmic bytes per domain and kernel
  std::vector<CycleGraph> cycles[2];            // cached solve-cycle graphs per side
  std::vector<IterGraph> iters;                 // cached whole-iteration graphs
  RunRecord *run = nullptr;                     // last multi-frame run (osmpm_batch_run)
  std::vector<void *> allocs;
};

namespace {

constexpr const char *kNoPlasticAdjoint =
    "the reverse mode has no derivative of the plastic projection (a material has a finite yield stress)";

osmpm_status fail(osmpm_ctx *c, osmpm_status s, const std::string &msg) {
  if (c) c->last_error = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                                            \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail((ctx), OSMPM_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

osmpm_status dalloc_bytes(osmpm_ctx *c, std::vector<void *> &list, void **p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return fail(c, OSMPM_E_NO_MEMORY, "hipMalloc failed");
  }
  list.push_back(*p);
  return OSMPM_OK;
}

template <typename T>
osmpm_status dalloc(osmpm_domain *d, T **p, size_t n) {
  void *q = nullptr;
  osmpm_status s = dalloc_bytes(d->ctx, d->allocs, &q, n * sizeof(T));
  *p = static_cast<T *>(q);
  return s;
}

osmpm_status ensure_pin(osmpm_ctx *c, size_t bytes) {
  if (c->h_pin_bytes >= bytes) return OSMPM_OK;
  if (c->h_pin) (void)hipHostFree(c->h_pin);
  c->h_pin = nullptr;
  c->h_pin_bytes = 0;
  const size_t nb = std::max<size_t>(bytes, 1 << 16);
  if (hipHostMalloc((void **)&c->h_pin, nb, hipHostMallocDefault) != hipSuccess)
    return fail(c, OSMPM_E_NO_MEMORY, "hipHostMalloc failed");
  c->h_pin_bytes = nb;
  return OSMPM_OK;
}

// ---------------------------------------------------------------- launches and profiling
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

// Appends a kernel node to the graph being built; the arguments are
// converted to the kernel's parameter types and copied by the runtime.
template <typename... P, typename... A>
void add_node(GraphBuild &gb, void (*kernel)(P...), dim3 grid, dim3 block, size_t shm, A... args) {
  std::tuple<P...> vals(static_cast<P>(args)...);
  void *ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
  std::apply(
      [&](auto &...v) {
        int i = 0;
        ((ptrs[i++] = static_cast<void *>(&v)), ...);
      },
      vals);
  hipKernelNodeParams np{};
  np.func = reinterpret_cast<void *>(kernel);
  np.gridDim = grid;
  np.blockDim = block;
  np.sharedMemBytes = (unsigned)shm;
  np.kernelParams = ptrs;
  np.extra = nullptr;
  hipGraphNode_t node = nullptr;
  const hipError_t e = hipGraphAddKernelNode(&node, gb.graph, gb.last ? &gb.last : nullptr, gb.last ? 1 : 0, &np);
  if (e != hipSuccess) {
    if (gb.err == hipSuccess) gb.err = e;
  } else {
    gb.last = node;
  }
}

// Every launch goes through here.  While a graph is being built the launch
// becomes a node.  With profiling on, an instrumented launch (which >= 0)
// carries start and stop timestamps on its own dispatch, so no extra packets
// sit between kernels.
template <typename F, typename... Args>
void launch(osmpm_ctx *c, int which, double bytes, int cg_iter, F kernel, dim3 grid, dim3 block, size_t shm,
            Args... args) {
  if (c->rec) {
    add_node(*c->rec, kernel, grid, block, shm, args...);
    return;
  }
  hipEvent_t a = nullptr, b = nullptr;
  if (c->prof && which >= 0) {
    a = prof_event(c);
    b = prof_event(c);
    if (!a || !b) a = b = nullptr;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shm, c->stream, a, b, 0, args...);
  if (a) c->pending.push_back({a, b, which, bytes, cg_iter});
}

// Folds completed timings into the counters (only after a stream
// synchronisation).  A CG launch with cycle index j is charged cg_bytes[j],
// the algorithmic bytes of the domains that iterated in it; launches in
// which every domain had finished (no entry, or zero) are dropped.  A span
// (the CG launches of one cycle between two events) counts its working
// launches and is charged their bytes and the whole span's time.
void prof_harvest(osmpm_ctx *c, const std::vector<double> *cg_bytes = nullptr) {
  for (const ProfPending &p : c->pending) {
    double bytes = p.bytes;
    int64_t n = 1;
    if (p.cg_iter >= 0) {
      bytes = (cg_bytes && p.cg_iter < (int)cg_bytes->size()) ? (*cg_bytes)[p.cg_iter] : 0.0;
    } else if (p.cg_iter == kCgSpan) {
      bytes = 0.0;
      n = 0;
      if (cg_bytes)
        for (double v : *cg_bytes)
          if (v > 0.0) {
            bytes += v;
            ++n;
          }
    }
    if (p.cg_iter != -1 && !(bytes > 0.0)) n = 0;
    if (n > 0) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        ProfSlot &sl = c->slots[p.which];
        sl.launches += n;
        sl.ms += ms;
        sl.bytes += bytes;
      }
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

// Algorithmic bytes of one domain in one launch: the data the operation must
// move once (particle arrays read or written, node arrays gathered, atomics
// counted as read + write), independent of caching.
double alg_bytes(int which, int D, double np, double nn, double tb) {
  const double ns = (D * D) * (D * D + 1) / 2.0;
  switch (which) {
    // nn: active nodes (m > 0) of the last P2G
    case OSMPM_K_CG_ITER:  // x, Atil per particle; per DOF r, w, s, u, p, del, diag and the mask read,
                           // p, s, r, u, del written, one w cleared, w accumulated (rmw); mass per node
      return np * (8.0 * D + tb * ns) + nn * (D * (tb * 15.0 + 1.0) + 8.0);
    case OSMPM_K_P2G:  // every particle array read once (pre-sort order) and written once (storage
                       // order): x, mass, vol, mat, id, flags; v, B, F; mass and momentum (rmw) per node
      return np * 2.0 * (8.0 * (D + 2.0) + 9.0 + tb * (D + 2.0 * D * D)) + nn * 16.0 * (1.0 + D);
    case OSMPM_K_G2P:  // x read and written, F read; v, B, F written; u gathered per node
      return np * (16.0 * D + tb * (D + 3.0 * D * D)) + nn * 8.0 * D;
    case OSMPM_K_GRAD_HESS:  // x, vol, mat, F read; Atil written; u read, gradient rmw, diagonal rmw
      return np * (8.0 * (D + 1.0) + 4.0 + tb * (D * D + ns)) + nn * (8.0 * 3.0 * D + tb * 2.0 * D);
    default:
      return 0.0;
  }
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

size_t lds_p2g(int D, int nreg) { return (size_t)nreg * (sizeof(long long) * (1 + kMaxGroups) + sizeof(double) * (1 + D)); }
size_t lds_grad(int D, int nreg) { return (size_t)nreg * sizeof(double) * 3 * D; }
size_t lds_hvp(int D, int nreg, size_t tb) { return (size_t)nreg * (sizeof(double) + tb) * D; }

double fixed_scale(const osmpm_domain *d) { return 4294967296.0 / d->m_ref; }
long long tau_fixed(const osmpm_domain *d) { return llrint(d->tau * fixed_scale(d)); }

// ---------------------------------------------------------------- groups
void group_free(osmpm_batch *G) {
  if (!G) return;
  osmpm_ctx *c = G->c;
  if (c) {
    (void)hipStreamSynchronize(c->stream);
    auto it = std::find(c->groups.begin(), c->groups.end(), G);
    if (it != c->groups.end()) c->groups.erase(it);
  }
  for (int s = 0; s < 2; ++s)
    for (CycleGraph &cgph : G->cycles[s])
      if (cgph.exec) (void)hipGraphExecDestroy(cgph.exec);
  for (IterGraph &ig : G->iters)
    if (ig.exec) (void)hipGraphExecDestroy(ig.exec);
  if (G->h_status) (void)hipHostFree(G->h_status);
  run_free(G->run);
  for (void *p : G->allocs) (void)hipFree(p);
  delete G;
}

// Per-domain partial-sum stride: the most workgroups any reduction of the
// domain uses.
int partial_stride(const osmpm_domain *d) {
  const int nd = d->g.nn * d->D;
  return std::max({node_blocks(nd), particle_blocks_host(d->cap), d->tg.nblocks, 2 * node_blocks(d->g.nn)}) + 8;
}

osmpm_status group_create(osmpm_ctx *c, int n, osmpm_domain *const *side0, osmpm_domain *const *side1,
                          osmpm_batch **out) {
  *out = nullptr;
  if (n < 1 || n > 1024 || !side0) return fail(c, OSMPM_E_INVALID_ARG, "group size must be 1..1024");
  auto *G = new osmpm_batch();
  G->c = c;
  G->uid = c->next_uid++;
  G->n = n;
  G->sides = side1 ? 2 : 1;
  G->D = side0[0] ? side0[0]->D : 2;
  G->precision = side0[0] ? side0[0]->precision : 0;
  for (int s = 0; s < G->sides; ++s) {
    osmpm_domain *const *src = s ? side1 : side0;
    for (int i = 0; i < n; ++i) {
      osmpm_domain *d = src[i];
      if (!d || d->ctx != c || d->D != G->D || d->precision != G->precision) {
        delete G;
        return fail(c, OSMPM_E_INVALID_ARG, "group members must share context, dimension and precision");
      }
      G->dom[s].push_back(d);
      G->stride = std::max(G->stride, partial_stride(d));
    }
    G->stamp_uid[s].assign(n, 0);
    G->stamp_ver[s].assign(n, 0);
    G->hdd[s].resize(n);
    G->act[s].assign(n, -1);
  }
  G->tb = G->dom[0][0]->tb;
  // status block layout
  size_t off = sizeof(StatusHdr);
  auto align = [](size_t v) { return (v + 63) & ~size_t(63); };
  G->off_amb = off;
  off = align(off + sizeof(int) * n);
  G->off_recv = off;
  off = align(off + sizeof(int) * 2 * n);
  G->off_res = off;
  off = align(off + sizeof(double) * 4 * n);
  G->off_ss = off;
  off = align(off + sizeof(SolveState) * 2 * n);
  G->off_cg = off;
  off = align(off + sizeof(CgState) * 2 * n);
  G->status_bytes = off;
  osmpm_status s = OSMPM_OK;
  void *p = nullptr;
  if (!s) s = dalloc_bytes(c, G->allocs, &p, G->status_bytes);
  if (!s) {
    G->status = static_cast<char *>(p);
    G->err = reinterpret_cast<int *>(G->status);
    G->n_amb = reinterpret_cast<int *>(G->status + G->off_amb);
    G->n_recv = reinterpret_cast<int *>(G->status + G->off_recv);
    G->res = reinterpret_cast<double *>(G->status + G->off_res);
    for (int sd = 0; sd < 2; ++sd) {
      G->ss[sd] = reinterpret_cast<SolveState *>(G->status + G->off_ss) + sd * n;
      G->cg[sd] = reinterpret_cast<CgState *>(G->status + G->off_cg) + sd * n;
    }
  }
  for (int sd = 0; sd < G->sides && !s; ++sd) {
    if (!s) s = dalloc_bytes(c, G->allocs, &p, sizeof(DomDesc) * n);
    G->dd[sd] = static_cast<DomDesc *>(p);
    if (!s) s = dalloc_bytes(c, G->allocs, &p, sizeof(int) * n);
    G->active[sd] = static_cast<int *>(p);
  }
  if (!s) s = dalloc_bytes(c, G->allocs, &p, sizeof(double) * (size_t)G->stride * kPartArrays * 2 * n);
  G->parts = static_cast<double *>(p);
  if (!s && hipMemsetAsync(G->status, 0, G->status_bytes, c->stream) != hipSuccess)
    s = fail(c, OSMPM_E_DEVICE, "hipMemsetAsync failed");
  if (!s && hipHostMalloc((void **)&G->h_status, G->status_bytes, hipHostMallocDefault) != hipSuccess)
    s = fail(c, OSMPM_E_NO_MEMORY, "hipHostMalloc failed");
  if (s) {
    group_free(G);
    return s;
  }
  c->groups.push_back(G);
  *out = G;
  return OSMPM_OK;
}

DomDesc make_desc(const osmpm_domain *d) {
  DomDesc x{};
  x.g = d->g;
  x.tg = d->tg;
  x.bc = d->bc;
  x.np = d->np;
  x.ndof = d->g.nn * d->D;
  x.nk = d->nk;
  x.cap = d->cap;
  x.scale = fixed_scale(d);
  x.tau_q = tau_fixed(d);
  x.Dinv = 4.0 * d->g.inv_dx * d->g.inv_dx;
  x.cur = d->d_cur;
  x.pb[0] = d->pb[0];
  x.pb[1] = d->pb[1];
  x.st = d->st;
  x.key = d->key;
  x.count = d->count;
  x.cell_start = d->cell_start;
  x.cursor = d->cursor;
  x.perm = d->perm;
  x.lperm = d->lperm;
  x.tcount = d->tcount;
  x.tl = d->tl;
  x.nlist = d->nlist;
  x.ncnt = d->ncnt;
  x.lcnt = d->lcnt;
  x.mu = d->mu;
  x.lam = d->lam;
  x.tau_y = d->tau_y;
  x.plastic = d->plastic ? 1 : 0;
  x.m = d->m;
  x.vn = d->vn;
  x.u = d->u;
  x.vbc = d->vbc;
  x.gg = d->gg;
  x.bcg = d->bcg;
  x.gamma = d->gamma;
  x.recv = d->recv;
  x.fr = d->fr;
  x.q_all = d->q_all;
  x.q_bnd = d->q_bnd;
  x.qg = d->qg;
  x.gd = d->gd;
  for (int k = 0; k < 2; ++k) {
    x.cr[k] = d->cr[k];
    x.cs[k] = d->cs[k];
  }
  for (int k = 0; k < 3; ++k) x.cw[k] = d->cw[k];
  x.cu = d->cu;
  x.cp = d->cp;
  x.del = d->del;
  x.Atil = d->Atil;
  x.pnum = d->pnum;
  x.pden = d->pden;
  x.w0 = d->w0;
  x.w1 = d->w1;
  x.w2 = d->w2;
  x.w3 = d->w3;
  x.flink = d->flink;
  x.warm = d->warm;
  x.warm_stride = d->g.nn * (d->D + 1) + 1;
  return x;
}

osmpm_status read_status(osmpm_batch *G);

// Uploads the descriptors of members whose configuration changed since the
// last upload and recomputes the launch extents.
osmpm_status group_sync(osmpm_batch *G) {
  osmpm_ctx *c = G->c;
  if (G->dead) return fail(c, OSMPM_E_STATE, "a domain of this batch was destroyed");
  for (int s = 0; s < G->sides; ++s) {
    bool changed = false;
    for (int i = 0; i < G->n; ++i) {
      osmpm_domain *d = G->dom[s][i];
      if (G->stamp_uid[s][i] == d->uid && G->stamp_ver[s][i] == d->version) continue;
      DomDesc x = make_desc(d);
      x.active = G->active[s] + i;
      x.ss = G->ss[s] + i;
      x.cg = G->cg[s] + i;
      double *base = G->parts + (size_t)((s * G->n + i) * kPartArrays) * G->stride;
      x.part_a = base;
      x.part_b = base + G->stride;
      x.part_cg = base + 2 * (size_t)G->stride;
      x.pstride = G->stride;
      G->hdd[s][i] = x;
      G->stamp_uid[s][i] = d->uid;
      G->stamp_ver[s][i] = d->version;
      changed = true;
    }
    if (!changed) continue;
    for (CycleGraph &cgph : G->cycles[s])  // launch extents may change
      if (cgph.exec) (void)hipGraphExecDestroy(cgph.exec);
    G->cycles[s].clear();
    for (IterGraph &ig : G->iters)
      if (ig.exec) (void)hipGraphExecDestroy(ig.exec);
    G->iters.clear();
    HIP_TRY(c, hipMemcpyAsync(G->dd[s], G->hdd[s].data(), sizeof(DomDesc) * G->n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    Ext E;
    for (int w = 0; w < OSMPM_K_COUNT; ++w) G->bytes[s][w].assign(G->n, 0.0);
    for (int i = 0; i < G->n; ++i) {
      const osmpm_domain *d = G->dom[s][i];
      const int nd = d->g.nn * d->D;
      E.max_np = std::max(E.max_np, d->np);
      E.max_nn = std::max(E.max_nn, d->g.nn);
      E.max_ndof = std::max(E.max_ndof, nd);
      E.max_nk = std::max(E.max_nk, d->nk);
      E.tile_blocks = std::max(E.tile_blocks, d->tg.nblocks);
      E.node_blocks = std::max(E.node_blocks, node_blocks(nd));
      E.part_blocks = std::max(E.part_blocks, particle_blocks_host(d->np));
      E.nn_blocks = std::max(E.nn_blocks, node_blocks(d->g.nn));
      E.lds_p2g = std::max(E.lds_p2g, lds_p2g(d->D, d->tg.nreg));
      E.lds_grad = std::max(E.lds_grad, lds_grad(d->D, d->tg.nreg));
      E.lds_hvp = std::max(E.lds_hvp, lds_hvp(d->D, d->tg.nreg, d->tb));
    }
    G->ext[s] = E;
  }
  if (c->prof) return read_status(G);  // byte counts from the last P2G's active nodes
  return OSMPM_OK;
}

// Sets the active flags of one side (a launch only when they change).
void set_active(osmpm_batch *G, int s, const std::vector<int> &want) {
  if (want == G->act[s]) return;
  FlagMask m{};
  for (int i = 0; i < G->n; ++i)
    if (want[i]) m.w[i >> 6] |= (uint64_t)1 << (i & 63);
  launch(G->c, -1, 0, -1, k_set_flags, dim3(blocks_for(G->n)), dim3(kBlock), 0, G->active[s], G->n, m);
  G->act[s] = want;
}

void set_all_active(osmpm_batch *G) {
  std::vector<int> one(G->n, 1);
  for (int s = 0; s < G->sides; ++s) set_active(G, s, one);
}

double active_bytes(const osmpm_batch *G, int s, int which) {
  double b = 0.0;
  for (int i = 0; i < G->n; ++i)
    if (G->act[s][i] == 1) b += G->bytes[s][which][i];
  return b;
}

// Device error of the status block last copied to the host (sticky: the
// word is never cleared).
osmpm_status status_error(osmpm_batch *G) {
  int err = 0;
  std::memcpy(&err, G->h_status, sizeof(int));
  return device_error(G->c, err);
}

const SolveState *h_ss(const osmpm_batch *G, int s) {
  return reinterpret_cast<const SolveState *>(G->h_status + G->off_ss) + s * G->n;
}

// Algorithmic bytes of the instrumented kernels for every domain of the
// group, from particle counts and the active-node counts of the last P2G as
// held by the host copy of the status block.
void refresh_bytes(osmpm_batch *G) {
  for (int s = 0; s < G->sides; ++s) {
    const SolveState *hs = h_ss(G, s);
    for (int w = 0; w < OSMPM_K_COUNT; ++w) G->bytes[s][w].resize(G->n, 0.0);
    for (int i = 0; i < G->n; ++i) {
      const osmpm_domain *d = G->dom[s][i];
      for (int w = 0; w < OSMPM_K_COUNT; ++w)
        G->bytes[s][w][i] = alg_bytes(w, d->D, d->np, hs[i].n_active, (double)d->tb);
    }
  }
}

// Copies the status block to its pinned host copy and waits.
osmpm_status read_status(osmpm_batch *G) {
  osmpm_ctx *c = G->c;
  osmpm_status s = check_launch(c);
  if (s) return s;
  HIP_TRY(c, hipMemcpyAsync(G->h_status, G->status, G->status_bytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->prof) refresh_bytes(G);
  return status_error(G);
}
const CgState *h_cg(const osmpm_batch *G, int s) {
  return reinterpret_cast<const CgState *>(G->h_status + G->off_cg) + s * G->n;
}
const int *h_int(const osmpm_batch *G, size_t off) { return reinterpret_cast<const int *>(G->h_status + off); }
const double *h_res(const osmpm_batch *G) { return reinterpret_cast<const double *>(G->h_status + G->off_res); }

// ---------------------------------------------------------------- work lists
// Live-tile list (from the bin offsets) and active-node list (from the node
// masses) of every active domain of side s; the CG launches map their
// workgroups onto them.
// (After a binning the tile scan builds the tile list, and after a P2G the
// final P2G pass has the node counts; these rebuild both for a restored
// binning and grid.)
void build_tile_list(osmpm_batch *G, int s) {
  launch(G->c, -1, 0, -1, k_tile_list, dim3(1, G->n), dim3(1024), 0, (const DomDesc *)G->dd[s]);
}
void build_node_list(osmpm_batch *G, int s, bool counted) {
  const Ext &E = G->ext[s];
  // the tile list of side s is rebuilt (binning or restore) before its node
  // list, so from here this group's status holds both counts
  for (int i = 0; i < G->n; ++i)
    if (G->act[s][i] == 1) G->dom[s][i]->lists_by = G->uid;
  if (!counted)
    launch(G->c, -1, 0, -1, k_node_count, dim3(blocks_for(E.max_nn), G->n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[s]);
  if (blocks_for(E.max_nn) > kNodeListDirect)
    launch(G->c, -1, 0, -1, k_node_scan, dim3(1, G->n), dim3(1024), 0, (const DomDesc *)G->dd[s]);
  launch(G->c, -1, 0, -1, k_node_list, dim3(blocks_for(E.max_nn), G->n), dim3(kBlock), 0, (const DomDesc *)G->dd[s]);
}

// ---------------------------------------------------------------- sort + P2G + G2P
// Stable counting sort of every active domain's particles by tile-major bin
// key (the storage permutation lperm; P2G gathers the particle arrays into
// the other buffer in that order); P2G targets are cleared.
template <int D, typename TB>
void sort_side(osmpm_batch *G, int s, int want_q) {
  osmpm_ctx *c = G->c;
  const Ext &E = G->ext[s];
  const DomDesc *dd = G->dd[s];
  const int n = G->n;
  const int pb = blocks_for(E.max_np);
  launch(c, -1, 0, -1, k_zero_grid, dim3(blocks_for(std::max(E.max_nk, E.max_ndof), 1024), n), dim3(kBlock), 0, dd,
         want_q);
  launch(c, -1, 0, -1, k_keys<D>, dim3(pb, n), dim3(kBlock), 0, dd, G->err);
  launch(c, -1, 0, -1, k_tile_sum, dim3(E.tile_blocks, n), dim3(kBlock), 0, dd);
  launch(c, -1, 0, -1, k_tile_scan, dim3(1, n), dim3(1024), 0, dd);
  launch(c, -1, 0, -1, k_cell_scan, dim3(E.tile_blocks, n), dim3(kBlock), 0, dd);
  launch(c, -1, 0, -1, k_scatter, dim3(pb, n), dim3(kBlock), 0, dd);
  launch(c, -1, 0, -1, k_cellsort, dim3(blocks_for(E.max_nk), n), dim3(kBlock), 0, dd);
  launch(c, -1, 0, -1, k_slot_layout, dim3(E.tile_blocks, n), dim3(kBlock), 0, dd);
}

template <int D, typename TB>
void p2g_side(osmpm_batch *G, int s, bool want_qall) {
  osmpm_ctx *c = G->c;
  int want_q = want_qall ? 1 : 0;
  for (int i = 0; i < G->n; ++i)
    if (G->act[s][i] == 1 && G->dom[s][i]->bc.n_groups > 0) want_q = 1;
  sort_side<D, TB>(G, s, want_q);
  const Ext &E = G->ext[s];
  if (want_q)
    launch(c, OSMPM_K_P2G, active_bytes(G, s, OSMPM_K_P2G), -1, k_p2g<D, TB, true>, dim3(E.tile_blocks, G->n),
           dim3(kBlock), E.lds_p2g, (const DomDesc *)G->dd[s], G->err);
  else
    launch(c, OSMPM_K_P2G, active_bytes(G, s, OSMPM_K_P2G), -1, k_p2g<D, TB, false>, dim3(E.tile_blocks, G->n),
           dim3(kBlock), E.lds_p2g, (const DomDesc *)G->dd[s], G->err);
  // P2G wrote the particles in storage order into the other buffer
  launch(c, -1, 0, -1, k_flip, dim3(blocks_for(G->n)), dim3(kBlock), 0, (const DomDesc *)G->dd[s], G->n);
  for (int i = 0; i < G->n; ++i)
    if (G->act[s][i] == 1) G->dom[s][i]->cur ^= 1;
  launch(c, -1, 0, -1, k_p2g_final<D>, dim3(blocks_for(E.max_nn), G->n), dim3(kBlock), 0, (const DomDesc *)G->dd[s]);
  build_node_list(G, s, true);
  for (int i = 0; i < G->n; ++i)
    if (G->act[s][i] == 1) {
      G->dom[s][i]->have_p2g = true;
      G->dom[s][i]->have_solve = false;
    }
  if (c->prof && read_status(G) == OSMPM_OK && !c->pending.empty()) {
    // charge the P2G just timed with the active nodes it produced
    for (auto it = c->pending.rbegin(); it != c->pending.rend(); ++it)
      if (it->which == OSMPM_K_P2G) {
        it->bytes = active_bytes(G, s, OSMPM_K_P2G);
        break;
      }
  }
}

template <int D, typename TB>
void g2p_side(osmpm_batch *G, int s, double dt) {
  const Ext &E = G->ext[s];
  launch(G->c, OSMPM_K_G2P, active_bytes(G, s, OSMPM_K_G2P), -1, k_g2p<D, TB>, dim3(blocks_for(E.max_np), G->n),
         dim3(kBlock), 0, (const DomDesc *)G->dd[s], dt, G->err);
  // any member with a yielding material (the kernel skips inactive and
  // elastic domains itself, so a recorded launch serves every active set)
  bool plastic = false;
  for (int i = 0; i < G->n; ++i)
    if (G->dom[s][i]->plastic) plastic = true;
  if (plastic)
    launch(G->c, -1, 0, -1, k_plastic_return<D, TB>, dim3(blocks_for(E.max_np), G->n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[s]);
}

template <int D, typename TB>
void copy_state_side(osmpm_batch *G, int s, int to_store) {
  const Ext &E = G->ext[s];
  launch(G->c, -1, 0, -1, k_copy_state<D, TB>, dim3(blocks_for(E.max_np), G->n), dim3(kBlock), 0,
         (const DomDesc *)G->dd[s], to_store);
}

// ---------------------------------------------------------------- implicit solve
// Newton-PCG-line-search on every active domain of side s.  The host queues
// cycles of [CG launches | line-search start | line-search round | step |
// gradient, Newton test, CG start] and reads the states after each cycle;
// each domain advances through its own phases on the device and skips the
// launches of phases it is not in.  The number of CG launch pairs of a cycle
// is sized from each domain's previous CG count.
template <int D, typename TB>
osmpm_status solve_side(osmpm_batch *G, int s, double dt, int use_schwarz, int vbc_buf, const osmpm_solve_opts *o,
                        std::vector<osmpm_solve_stats> *out, int warm_slot = -1, int warm_use = 0) {
  osmpm_ctx *c = G->c;
  const Ext &E = G->ext[s];
  const DomDesc *dd = G->dd[s];
  const int n = G->n;
  const dim3 blk(kBlock);
  const int wstart = (warm_slot >= 0 && warm_use) ? warm_slot : -1;
  osmpm_status st;
  // Launch sizes of the tangent pass and the CG iteration.  Their workgroups
  // past the live-tile slots and the active-DOF blocks leave at once, but on
  // a grid that is mostly empty tiles those are most of the launch (on the
  // fine domain of the hinge at the paper's resolution, 1.9M of 2.2M
  // workgroups, 2 ms of each 12 ms CG iteration).  Above kSizedLaunch tile
  // workgroups the solve first reads the status (the live-tile and
  // active-node counts of the last binning and P2G, which no solve kernel
  // changes) and sizes both launches to the largest working count of its
  // domains, by the formula the kernels use.  The counts live in the status
  // of the group that built the lists, so a solve through another group
  // keeps the full launches (the entry points bin a domain in the group that
  // then solves it, and a solve after G2P without a new binning is refused,
  // so this only guards the sequencing), as does a recorded solve, whose
  // sizes must not depend on the state.
  int grid_t = E.tile_blocks, grid_cg = E.tile_blocks;
  bool own_counts = true;  // this group built every solving domain's work lists
  for (int i = 0; i < n; ++i)
    if (G->act[s][i] == 1 && G->dom[s][i]->lists_by != G->uid) own_counts = false;
  if (!c->rec && own_counts && E.tile_blocks > kSizedLaunch) {
    if ((st = read_status(G))) return st;
    const SolveState *h = h_ss(G, s);
    grid_t = grid_cg = 1;
    for (int i = 0; i < n; ++i)
      if (G->act[s][i] == 1) {
        const osmpm_domain *d = G->dom[s][i];
        grid_t = std::max(grid_t, std::min(((h[i].n_tiles_live + 7) / 8) * 8, d->tg.nblocks));
        grid_cg = std::max(grid_cg, cg_work_blocks(h[i].n_tiles_live, h[i].n_active * d->D, d->tg.nblocks));
      }
  }
  launch(c, -1, 0, -1, k_bc_init<D, TB>, dim3(E.node_blocks, n), blk, 0, dd, dt, use_schwarz, vbc_buf, wstart);
  launch(c, -1, 0, -1, k_solve_begin, dim3(1, n), blk, 0, dd, dt, wstart);
  const double bg = active_bytes(G, s, OSMPM_K_GRAD_HESS);
  auto grad_phase = [&]() {
    launch(c, OSMPM_K_GRAD_HESS, bg, -1, k_grad_hess<D, TB>, dim3(grid_t, n), blk, E.lds_grad, dd,
           (int)o->project_psd, G->err);
    launch(c, -1, 0, -1, k_grad_node<D, TB>, dim3(E.node_blocks, n), blk, 0, dd, dt, o->gravity[0], o->gravity[1],
           o->gravity[2]);
    launch(c, -1, 0, -1, k_cg_init<D, TB>, dim3(E.node_blocks, n), blk, 0, dd, 1, o->newton_rtol, o->newton_atol,
           (int)o->max_newton, o->forcing);
  };
  grad_phase();
  // Split CG scalars (k_cg_reduce after each iteration) when the fused form's
  // pass of every workgroup over all partial sums would read more than a
  // dependent launch costs (measured: the 3D fold gains, a 64-scene 2D batch
  // at ~60 MB does not): sum over domains of 24 B x workgroups^2, with the
  // working workgroups estimated from the live tiles and active nodes of the
  // last status read (the tile blocks before any).
  double partial_reads = 0.0;
  const SolveState *hss = h_ss(G, s);
  for (int i = 0; i < n; ++i)
    if (G->act[s][i] == 1) {
      const osmpm_domain *d = G->dom[s][i];
      double w = d->tg.nblocks;
      if (hss[i].n_tiles_live > 0) {
        const double nt8 = 8.0 * ((hss[i].n_tiles_live + 7) / 8);
        const double nown = std::ceil((double)hss[i].n_active * d->D / kBlock);
        w = std::min<double>(d->tg.nblocks, std::max(nt8, nown));
      }
      partial_reads += 24.0 * w * w;
    }
  const int split = c->cg_split >= 0 ? c->cg_split : (partial_reads > 128e6 ? 1 : 0);
  std::vector<int> hint(n), prev_phase(n, kPhaseCgInit), prev_iter(n, 0), prev_total(n, 0);
  for (int i = 0; i < n; ++i) hint[i] = G->dom[s][i]->cg_hint;
  const long max_cycles = (long)(o->max_newton + 1) * ((o->max_cg + 4) / 4 + o->max_ls + 3) + 8;
  if (c->rec) {
    // Recorded into a whole-iteration graph (fixed-schedule solves: one
    // Newton step of exactly max_cg CG iterations, no halving): one cycle
    // of max_cg + 2 CG launches ends every domain's solve, so no state is
    // read back; the counts go to the device totals.
    int b = o->max_cg + 2;
    b += b & 1;
    for (int j = 0; j < b; ++j) {
      launch(c, -1, 0, -1, k_cg_iter<D, TB>, dim3(E.tile_blocks, n), blk, E.lds_hvp, dd, j & 1, dt, o->cg_rtol,
             (int)o->max_cg, split);
      if (split)
        launch(c, -1, 0, -1, k_cg_reduce, dim3(cg_reduce_blocks(E.tile_blocks), n), blk, 0, dd, j & 1, o->cg_rtol,
               (int)o->max_cg);
    }
    launch(c, -1, 0, -1, k_delta_energy<D, TB>, dim3(E.part_blocks + E.node_blocks, n), blk, 0, dd, dt,
           o->gravity[0], o->gravity[1], o->gravity[2]);
    launch(c, -1, 0, -1, k_ls_check, dim3(1, n), blk, 0, dd, (int)o->max_ls);
    grad_phase();
    if (warm_slot >= 0)
      launch(c, -1, 0, -1, k_warm_keep, dim3(E.node_blocks, n), blk, 0, dd, warm_slot, warm_use ? 0 : 1);
    launch(c, -1, 0, -1, k_solve_tally, dim3(1, n), blk, 0, dd, 0);
    return OSMPM_OK;
  }
  // A warm-started solve often passes its first Newton test: one status
  // read then costs less than a cycle of launches that would find every
  // domain done.
  bool skip_cycles = false;
  if (wstart >= 0 && !c->graphs) {
    if ((st = read_status(G))) return st;
    const SolveState *h0 = h_ss(G, s);
    skip_cycles = true;
    for (int i = 0; i < n; ++i)
      if (G->act[s][i] == 1 && h0[i].phase != kPhaseDone) skip_cycles = false;
  }
  for (long cyc = 0; !skip_cycles; ++cyc) {
    if (cyc > max_cycles) return fail(c, OSMPM_E_STATE, "implicit solve did not terminate");
    // launches wanted this cycle: a fresh CG of n iterations takes n + 2
    // (the product of u_0, n steps, the stop test), a running one the rest,
    // at least 4; none when no domain is in CG (a line-search halving only)
    int b = 0;
    for (int i = 0; i < n; ++i) {
      if (G->act[s][i] != 1) continue;
      if (prev_phase[i] == kPhaseCgInit) b = std::max({b, 4, hint[i] + 2});
      if (prev_phase[i] == kPhaseCg) b = std::max({b, 4, hint[i] - prev_iter[i] + 1});
    }
    b = std::min(b, o->max_cg + 2);
    b += b & 1;  // even, so every cycle starts at parity 0
    if (c->graphs && !c->prof) b = (b + 3) & ~3;  // fewer distinct cycle graphs
    auto cycle = [&]() {
      // With profiling on, the cycle's back-to-back CG launches are timed as
      // one span between two events: an event pair on every launch would add
      // a fixed cost of about 2 us to each measured duration.
      hipEvent_t sa = nullptr, sb = nullptr;
      if (c->prof && !c->rec) {
        sa = prof_event(c);
        sb = prof_event(c);
        if (sa && sb && hipEventRecord(sa, c->stream) != hipSuccess) sa = nullptr;
      }
      for (int j = 0; j < b; ++j) {
        launch(c, sa ? -1 : OSMPM_K_CG_ITER, 0.0, j, k_cg_iter<D, TB>, dim3(grid_cg, n), blk, E.lds_hvp, dd,
               j & 1, dt, o->cg_rtol, (int)o->max_cg, split);
        if (split)
          launch(c, -1, 0, -1, k_cg_reduce, dim3(cg_reduce_blocks(grid_cg), n), blk, 0, dd, j & 1,
                 o->cg_rtol, (int)o->max_cg);
      }
      if (sa && sb && hipEventRecord(sb, c->stream) == hipSuccess)
        c->pending.push_back({sa, sb, OSMPM_K_CG_ITER, 0.0, kCgSpan});
      launch(c, -1, 0, -1, k_delta_energy<D, TB>, dim3(E.part_blocks + E.node_blocks, n), blk, 0, dd, dt,
             o->gravity[0], o->gravity[1], o->gravity[2]);
      launch(c, -1, 0, -1, k_ls_check, dim3(1, n), blk, 0, dd, (int)o->max_ls);
      grad_phase();
    };
    if (c->graphs && !c->prof) {
      // replay the cycle (its launches and the status copy) as one graph
      CycleGraph *cg = nullptr;
      for (CycleGraph &x : G->cycles[s])
        if (x.b == b && x.grid_t == grid_t && x.grid_cg == grid_cg && x.dt == dt &&
            std::memcmp(&x.o, o, sizeof(osmpm_solve_opts)) == 0)
          cg = &x;
      if (!cg) {
        GraphBuild gb;
        HIP_TRY(c, hipGraphCreate(&gb.graph, 0));
        c->rec = &gb;
        cycle();
        c->rec = nullptr;
        hipGraphNode_t cp = nullptr;
        if (gb.err == hipSuccess)
          gb.err = hipGraphAddMemcpyNode1D(&cp, gb.graph, gb.last ? &gb.last : nullptr, gb.last ? 1 : 0,
                                           G->h_status, G->status, G->status_bytes, hipMemcpyDeviceToHost);
        hipGraphExec_t ex = nullptr;
        if (gb.err == hipSuccess) gb.err = hipGraphInstantiate(&ex, gb.graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gb.graph);
        if (gb.err != hipSuccess)
          return fail(c, OSMPM_E_DEVICE, std::string("solve cycle graph: ") + hipGetErrorString(gb.err));
        CycleGraph x;
        x.b = b;
        x.grid_t = grid_t;
        x.grid_cg = grid_cg;
        x.dt = dt;
        x.o = *o;
        x.exec = ex;
        G->cycles[s].push_back(x);
        cg = &G->cycles[s].back();
      }
      if ((st = check_launch(c))) return st;
      HIP_TRY(c, hipGraphLaunch(cg->exec, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      if ((st = status_error(G))) return st;
    } else {
      cycle();
      if ((st = read_status(G))) return st;
    }
    const SolveState *hs = h_ss(G, s);
    const CgState *hc = h_cg(G, s);
    std::vector<double> cg_bytes(b, 0.0);
    bool all_done = true;
    for (int i = 0; i < n; ++i) {
      if (G->act[s][i] != 1) continue;
      const bool was_cg = prev_phase[i] == kPhaseCgInit || prev_phase[i] == kPhaseCg;
      const int start = prev_phase[i] == kPhaseCg ? prev_iter[i] : 0;
      int did = 0;
      const int extra = prev_phase[i] == kPhaseCgInit ? 1 : 0;  // the product of u_0
      if (was_cg && hs[i].phase != kPhaseCg) {  // a CG finished in this cycle
        const int cnt = hs[i].cg_iters - prev_total[i];
        hint[i] = cnt;
        did = cnt - start + 1 + extra;
      } else if (was_cg) {
        did = hc[i].iter - start + extra;
      }
      for (int j = 0; j < std::min(did, b); ++j) cg_bytes[j] += G->bytes[s][OSMPM_K_CG_ITER][i];
      prev_phase[i] = hs[i].phase;
      prev_iter[i] = hc[i].iter;
      prev_total[i] = hs[i].cg_iters;
      if (hs[i].phase != kPhaseDone) all_done = false;
    }
    prof_harvest(c, &cg_bytes);
    if (all_done) break;
  }
  if (warm_slot >= 0)
    launch(c, -1, 0, -1, k_warm_keep, dim3(E.node_blocks, n), blk, 0, dd, warm_slot, warm_use ? 0 : 1);
  const SolveState *hs = h_ss(G, s);
  if (out) out->assign(n, osmpm_solve_stats{});
  for (int i = 0; i < n; ++i) {
    if (G->act[s][i] != 1) continue;
    G->dom[s][i]->cg_hint = std::max(hint[i], 1);
    G->dom[s][i]->have_solve = true;
    if (out) {
      osmpm_solve_stats &r = (*out)[i];
      r.newton_iters = hs[i].newton_iters;
      r.cg_iters = hs[i].cg_iters;
      r.ls_halvings = hs[i].ls_halvings;
      r.converged = hs[i].converged;
      r.ls_failed = hs[i].ls_failed;
      r.gnorm0 = hs[i].gnorm0;
      r.gnorm = hs[i].gnorm;
    }
  }
  return OSMPM_OK;
}

// ---------------------------------------------------------------- interface (two-sided groups)
template <int D>
void interface_group(osmpm_batch *G) {
  osmpm_ctx *c = G->c;
  const int n = G->n;
  for (int s = 0; s < 2; ++s) {
    launch(c, -1, 0, -1, k_qbnd<D>, dim3(blocks_for(G->ext[s].max_np), n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[s]);
    launch(c, -1, 0, -1, k_gamma, dim3(blocks_for(G->ext[s].max_nn), n), dim3(kBlock), 0, (const DomDesc *)G->dd[s]);
  }
  launch(c, -1, 0, -1, k_fill<int>, dim3(blocks_for(n)), dim3(kBlock), 0, (int64_t)n, 0, G->n_amb);
  launch(c, -1, 0, -1, k_arbitrate<D>, dim3(blocks_for(G->ext[0].max_nn), n), dim3(kBlock), 0,
         (const DomDesc *)G->dd[0], (const DomDesc *)G->dd[1], G->n_amb);
}

// Receiver counts of both sides into the status block (after arbitration).
template <int D>
void count_recv(osmpm_batch *G) {
  for (int s = 0; s < 2; ++s)
    launch(G->c, -1, 0, -1, k_count_recv, dim3(1, G->n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[s], G->n_recv + s * G->n);
}

// Pi_{S->B} into B's work buffer `which` (or out_ext when which < 0).
template <int D>
void project_group(osmpm_batch *G, double eps_tol, const double *vS_ext, int which, double *out_ext) {
  osmpm_ctx *c = G->c;
  const int n = G->n;
  launch(c, -1, 0, -1, k_zero_proj, dim3(blocks_for(G->ext[0].max_ndof, 1024), n), dim3(kBlock), 0,
         (const DomDesc *)G->dd[0]);
  launch(c, -1, 0, -1, k_project_scatter<D>, dim3(blocks_for(G->ext[1].max_nn), n), dim3(kBlock), 0,
         (const DomDesc *)G->dd[1], (const DomDesc *)G->dd[0], vS_ext, G->err);
  launch(c, -1, 0, -1, k_project_final<D>, dim3(blocks_for(G->ext[0].max_nn), n), dim3(kBlock), 0,
         (const DomDesc *)G->dd[0], eps_tol, which, out_ext);
}

// I_{B->S} from B's buffer src (or vB_ext) into S's buffer dst (or out_ext).
template <int D>
void interp_group(osmpm_batch *G, int src, const double *vB_ext, int dst, double *out_ext) {
  launch(G->c, -1, 0, -1, k_interp<D>, dim3(blocks_for(G->ext[1].max_nn), G->n), dim3(kBlock), 0,
         (const DomDesc *)G->dd[0], (const DomDesc *)G->dd[1], src, vB_ext, dst, out_ext, G->err);
}

// Relative interface changes r = |a - b| / |a| over each domain's receivers
// (Eq. convergence_residuals), reduced on the device into the status block.
template <int D>
void resid_side(osmpm_batch *G, int s, int a_buf, int b_buf) {
  osmpm_ctx *c = G->c;
  launch(c, -1, 0, -1, k_resid<D>, dim3(G->ext[s].nn_blocks, G->n), dim3(kBlock), 0, (const DomDesc *)G->dd[s],
         a_buf, b_buf);
  launch(c, -1, 0, -1, k_resid_final, dim3(1, G->n), dim3(kBlock), 0, (const DomDesc *)G->dd[s],
         G->res + 2 * s * G->n);
}

// Adds one implicit solve's counts to a frame's statistics of side B or S.
void add_stats(osmpm_schwarz_stats &st, bool fine, const osmpm_solve_stats &s) {
  (fine ? st.newton_S : st.newton_B) += s.newton_iters;
  (fine ? st.cg_S : st.cg_B) += s.cg_iters;
  (fine ? st.ls_S : st.ls_B) += s.ls_halvings;
  (fine ? st.unconv_S : st.unconv_B) += !s.converged;
  (fine ? st.lsfail_S : st.lsfail_B) += s.ls_failed;
}

// Warm-start slots of every domain of side s of a group (n_slots each),
// allocated or grown on first use; descriptors are re-uploaded when a
// buffer changes.
osmpm_status ensure_warm(osmpm_batch *G, int s, int n_slots) {
  bool changed = false;
  for (int i = 0; i < G->n; ++i) {
    osmpm_domain *d = G->dom[s][i];
    if (d->warm_slots >= n_slots) continue;
    if (d->warm) {
      (void)hipStreamSynchronize(d->ctx->stream);
      auto it = std::find(d->allocs.begin(), d->allocs.end(), (void *)d->warm);
      if (it != d->allocs.end()) d->allocs.erase(it);
      (void)hipFree(d->warm);
      d->warm = nullptr;
      d->warm_slots = 0;
    }
    const size_t stride = (size_t)d->g.nn * (d->D + 1) + 1;
    osmpm_status st = dalloc(d, &d->warm, stride * n_slots);
    if (st) return st;
    d->warm_slots = n_slots;
    d->version += 1;
    changed = true;
  }
  return changed ? group_sync(G) : OSMPM_OK;
}

// One global frame of Alg. 1 for every pair of a two-sided group.  Work
// buffer roles: on B, Pi data of the current and the next iteration alternate
// between w0 and w1, and w2 holds v_B^(k+1); on S, w0 holds I(v_B^n), and the
// new and previous I(v_B^(k+1)) alternate between w1 and w2.  A pair whose
// residuals pass the test leaves the group's launches; the coarse G2P runs
// for all pairs at the end.
template <int D, typename TB>
osmpm_status schwarz_group(osmpm_batch *G, double dT, const osmpm_schwarz_opts *o, osmpm_schwarz_stats *out) {
  osmpm_ctx *c = G->c;
  const int n = G->n;
  const int M = o->M;
  const double dt = dT / (double)M;
  osmpm_status s;
  if ((s = group_sync(G))) return s;
  const bool warm = o->warm_start != 0;
  if (warm && ((s = ensure_warm(G, 0, 1)) || (s = ensure_warm(G, 1, M)))) return s;
  std::vector<osmpm_schwarz_stats> st(n);
  set_all_active(G);
  // frame start: the fine state is stored, both grids built, the
  // interface sets formed, and the first iterate's coarse data projected
  copy_state_side<D, TB>(G, 1, 1);
  p2g_side<D, TB>(G, 0, true);
  p2g_side<D, TB>(G, 1, true);
  interface_group<D>(G);
  int piB = 0, piB_next = 1, iS_new = 1, iS_prev = 2;
  project_group<D>(G, o->eps_tol, nullptr, piB, nullptr);
  interp_group<D>(G, kBufVn, nullptr, iS_prev, nullptr);
  std::vector<int> live(n, 1);
  std::vector<osmpm_solve_stats> ss;
  // One Schwarz iteration's launches; while a graph is being recorded
  // (c->rec) the solves take their fixed schedule and report no counts.
  auto iteration = [&](int k) -> osmpm_status {
    osmpm_status r;
    const bool rec = c->rec != nullptr;
    // the coarse solve over dT takes buffer piB on its receivers
    if ((r = solve_side<D, TB>(G, 0, dT, 1, piB, &o->coarse, &ss, warm ? 0 : -1, k > 0))) return r;
    if (!rec)
      for (int i = 0; i < n; ++i)
        if (live[i]) add_stats(st[i], false, ss[i]);
    launch(c, -1, 0, -1, k_vel_from_u<D>, dim3(blocks_for(G->ext[0].max_nn), n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[0], dT);
    // the fine domains restart from the stored state and take M sub-steps
    // driven by the temporal interpolation of the two coarse endpoints
    copy_state_side<D, TB>(G, 1, 0);
    p2g_side<D, TB>(G, 1, false);
    interp_group<D>(G, kBufVn, nullptr, 0, nullptr);
    interp_group<D>(G, 2, nullptr, iS_new, nullptr);
    for (int m = 1; m <= M; ++m) {
      launch(c, -1, 0, -1, k_temporal<D>, dim3(blocks_for(G->ext[1].max_ndof, 1024), n), dim3(kBlock), 0,
             (const DomDesc *)G->dd[1], (double)m / (double)M, 0, iS_new);
      if ((r = solve_side<D, TB>(G, 1, dt, 1, kBufVbc, &o->fine, &ss, warm ? m - 1 : -1, k > 0))) return r;
      if (!rec)
        for (int i = 0; i < n; ++i)
          if (live[i]) add_stats(st[i], true, ss[i]);
      g2p_side<D, TB>(G, 1, dt);
      p2g_side<D, TB>(G, 1, false);
    }
    // the projection for iteration k + 1 and the interface changes
    project_group<D>(G, o->eps_tol, nullptr, piB_next, nullptr);
    resid_side<D>(G, 0, piB_next, piB);
    resid_side<D>(G, 1, iS_new, iS_prev);
    return OSMPM_OK;
  };
  // Whole iterations as graphs: both solves must have a fixed schedule, so
  // that an iteration is a fixed launch sequence (the Newton and line-search
  // decisions of adaptive solves are taken on the host between cycles, and
  // HIP graphs here have no conditional nodes).
  auto fixed = [](const osmpm_solve_opts &so) {
    return so.max_newton == 1 && so.max_ls == 0 && so.cg_rtol == 0.0 && so.max_cg >= 1;
  };
  const bool whole = c->graphs >= 2 && !c->prof && fixed(o->coarse) && fixed(o->fine);
  std::vector<int> prev_tally(whole ? 10 * n : 0, 0);
  if (whole)
    for (int sd = 0; sd < 2; ++sd)
      launch(c, -1, 0, -1, k_solve_tally, dim3(1, n), dim3(kBlock), 0, (const DomDesc *)G->dd[sd], 1);
  for (int k = 0; k < o->k_max; ++k) {
    if (whole) {
      const int cls = k == 0 ? 0 : 1 + (k & 1);
      IterGraph *ig = nullptr;
      for (IterGraph &x : G->iters)
        if (x.cls == cls && x.dT == dT && std::memcmp(&x.o, o, sizeof(osmpm_schwarz_opts)) == 0) ig = &x;
      if (!ig) {
        // recorded now and launched below; the host mirrors of the buffer
        // parity were advanced while recording
        GraphBuild gb;
        HIP_TRY(c, hipGraphCreate(&gb.graph, 0));
        c->rec = &gb;
        s = iteration(k);
        c->rec = nullptr;
        hipGraphNode_t cp = nullptr;
        if (!s && gb.err == hipSuccess)
          gb.err = hipGraphAddMemcpyNode1D(&cp, gb.graph, gb.last ? &gb.last : nullptr, gb.last ? 1 : 0,
                                           G->h_status, G->status, G->status_bytes, hipMemcpyDeviceToHost);
        hipGraphExec_t ex = nullptr;
        if (!s && gb.err == hipSuccess) gb.err = hipGraphInstantiate(&ex, gb.graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gb.graph);
        if (s) return s;
        if (gb.err != hipSuccess)
          return fail(c, OSMPM_E_DEVICE, std::string("Schwarz iteration graph: ") + hipGetErrorString(gb.err));
        IterGraph x;
        x.cls = cls;
        x.dT = dT;
        x.o = *o;
        x.exec = ex;
        G->iters.push_back(x);
        ig = &G->iters.back();
      } else {
        // a replay flips the particle buffers of every active fine domain
        // once per fine P2G (1 + M of them)
        if ((M + 1) & 1)
          for (int i = 0; i < n; ++i)
            if (G->act[1][i] == 1) G->dom[1][i]->cur ^= 1;
        for (int i = 0; i < n; ++i)
          if (G->act[1][i] == 1) {
            G->dom[1][i]->have_p2g = true;
            G->dom[1][i]->have_solve = false;
          }
      }
      if ((s = check_launch(c))) return s;
      HIP_TRY(c, hipGraphLaunch(ig->exec, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      if ((s = status_error(G))) return s;
      // the solves' counts of this iteration from the device totals
      for (int sd = 0; sd < 2; ++sd) {
        const SolveState *hs = h_ss(G, sd);
        for (int i = 0; i < n; ++i) {
          int *pv = &prev_tally[(sd * n + i) * 5];
          if (live[i]) {
            osmpm_schwarz_stats &q = st[i];
            const int *t = hs[i].tally;
            (sd ? q.newton_S : q.newton_B) += t[0] - pv[0];
            (sd ? q.cg_S : q.cg_B) += t[1] - pv[1];
            (sd ? q.ls_S : q.ls_B) += t[2] - pv[2];
            (sd ? q.unconv_S : q.unconv_B) += t[3] - pv[3];
            (sd ? q.lsfail_S : q.lsfail_B) += t[4] - pv[4];
          }
          for (int j = 0; j < 5; ++j) pv[j] = hs[i].tally[j];
        }
      }
    } else {
      if ((s = iteration(k))) return s;
      if ((s = read_status(G))) return s;
    }
    const double *res = h_res(G);
    std::swap(piB, piB_next);
    std::swap(iS_new, iS_prev);
    bool any = false;
    for (int i = 0; i < n; ++i) {
      if (!live[i]) continue;
      const double rB = std::sqrt(res[2 * i]) / std::max(std::sqrt(res[2 * i + 1]), 1e-30);
      const double rS = std::sqrt(res[2 * n + 2 * i]) / std::max(std::sqrt(res[2 * n + 2 * i + 1]), 1e-30);
      st[i].r_B = rB;
      st[i].r_S = rS;
      st[i].iters = k + 1;
      if (rB <= o->eps_conv && rS <= o->eps_conv) {
        st[i].converged = 1;
        live[i] = 0;
      } else {
        any = true;
      }
    }
    if (!any) break;
    set_active(G, 0, live);
    set_active(G, 1, live);
  }
  // every pair's coarse particles move with its last coarse solution
  set_all_active(G);
  g2p_side<D, TB>(G, 0, dT);
  count_recv<D>(G);
  if ((s = read_status(G))) return s;
  const int *amb = h_int(G, G->off_amb);
  const int *nrecv = h_int(G, G->off_recv);
  for (int i = 0; i < n; ++i) {
    st[i].n_amb = amb[i];
    st[i].n_recv_B = nrecv[i];
    st[i].n_recv_S = nrecv[n + i];
    if (out) out[i] = st[i];
  }
  return OSMPM_OK;
}

// Boundary sets of the coarse domain (once) and of every fine domain, and
// the arbitration of every fine domain against the coarse one (each copy of
// the coarse domain on side 0 meets its own fine domain).
template <int D>
void interface_multi(osmpm_batch *G, const std::vector<int> &b_one) {
  osmpm_ctx *c = G->c;
  const int n = G->n;
  set_active(G, 0, b_one);
  for (int s = 0; s < 2; ++s) {
    launch(c, -1, 0, -1, k_qbnd<D>, dim3(blocks_for(G->ext[s].max_np), n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[s]);
    launch(c, -1, 0, -1, k_gamma, dim3(blocks_for(G->ext[s].max_nn), n), dim3(kBlock), 0, (const DomDesc *)G->dd[s]);
  }
  launch(c, -1, 0, -1, k_fill<int>, dim3(blocks_for(n)), dim3(kBlock), 0, (int64_t)n, 0, G->n_amb);
  set_active(G, 0, std::vector<int>(n, 1));
  launch(c, -1, 0, -1, k_arbitrate<D>, dim3(blocks_for(G->ext[0].max_nn), n), dim3(kBlock), 0,
         (const DomDesc *)G->dd[0], (const DomDesc *)G->dd[1], G->n_amb);
  set_active(G, 0, b_one);
}

// One frame of Alg. 1 for one coarse domain and the k = G->n disjoint fine
// domains of a multi group (readings as for the oracle's multi-domain frame):
// coarse work runs on the first copy of the coarse domain only; the
// projection scatters every fine domain into the coarse sums; each fine
// domain is interpolated from the same coarse solution and sub-cycled (all of
// them in the same launches); r_S is taken over the receivers of all fine
// domains together, and the frame ends when both residuals pass.
template <int D, typename TB>
osmpm_status schwarz_multi(osmpm_batch *G, double dT, const osmpm_schwarz_opts *o, osmpm_schwarz_stats *out) {
  osmpm_ctx *c = G->c;
  const int n = G->n;
  const int M = o->M;
  const double dt = dT / (double)M;
  osmpm_status s;
  if ((s = group_sync(G))) return s;
  const bool warm = o->warm_start != 0;
  // the fine domains keep every sub-step's solution (the warm-start slots):
  // linked receivers of overlapping regions read them
  if ((warm && (s = ensure_warm(G, 0, 1))) || (s = ensure_warm(G, 1, M))) return s;
  osmpm_schwarz_stats st{};
  std::vector<int> b_one(n, 0), all(n, 1);
  b_one[0] = 1;
  set_active(G, 0, b_one);
  set_active(G, 1, all);
  // frame start: fine states stored, all grids built, interface sets
  copy_state_side<D, TB>(G, 1, 1);
  p2g_side<D, TB>(G, 0, true);
  p2g_side<D, TB>(G, 1, true);
  interface_multi<D>(G, b_one);
  if (n > 1) {
    launch(c, -1, 0, -1, k_fine_arbitrate<D>, dim3(blocks_for(G->ext[1].max_nn), n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[1], n, G->n_amb);
    launch(c, -1, 0, -1, k_fine_links<D>, dim3(blocks_for(G->ext[1].max_nn), n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[1], n);
  }
  int piB = 0, piB_next = 1, iS_new = 1, iS_prev = 2;
  project_group<D>(G, o->eps_tol, nullptr, piB, nullptr);
  interp_group<D>(G, kBufVn, nullptr, iS_prev, nullptr);
  std::vector<osmpm_solve_stats> ss;
  for (int k = 0; k < o->k_max; ++k) {
    // the coarse solve over dT takes buffer piB on its receivers
    if ((s = solve_side<D, TB>(G, 0, dT, 1, piB, &o->coarse, &ss, warm ? 0 : -1, k > 0))) return s;
    add_stats(st, false, ss[0]);
    launch(c, -1, 0, -1, k_vel_from_u<D>, dim3(blocks_for(G->ext[0].max_nn), n), dim3(kBlock), 0,
           (const DomDesc *)G->dd[0], dT);
    // every fine domain restarts from its stored state and is sub-cycled
    copy_state_side<D, TB>(G, 1, 0);
    p2g_side<D, TB>(G, 1, false);
    interp_group<D>(G, kBufVn, nullptr, 0, nullptr);
    interp_group<D>(G, 2, nullptr, iS_new, nullptr);
    for (int m = 1; m <= M; ++m) {
      launch(c, -1, 0, -1, k_temporal<D>, dim3(blocks_for(G->ext[1].max_ndof, 1024), n), dim3(kBlock), 0,
             (const DomDesc *)G->dd[1], (double)m / (double)M, 0, iS_new);
      if (n > 1 && k > 0)  // linked receivers: the donors' sub-step m of the previous iteration
        launch(c, -1, 0, -1, k_fine_link_apply<D>, dim3(blocks_for(G->ext[1].max_nn), n), dim3(kBlock), 0,
               (const DomDesc *)G->dd[1], m - 1, dt, -1);
      if ((s = solve_side<D, TB>(G, 1, dt, 1, kBufVbc, &o->fine, &ss, m - 1, warm && k > 0))) return s;
      for (int i = 0; i < n; ++i) add_stats(st, true, ss[i]);
      g2p_side<D, TB>(G, 1, dt);
      p2g_side<D, TB>(G, 1, false);
    }
    // linked receivers' data for the residual: the donors' end-of-frame
    // velocity (sub-step M) of this iteration
    if (n > 1)
      launch(c, -1, 0, -1, k_fine_link_apply<D>, dim3(blocks_for(G->ext[1].max_nn), n), dim3(kBlock), 0,
             (const DomDesc *)G->dd[1], M - 1, dt, iS_new);
    // the projection for iteration k + 1 and the changes over all interfaces
    project_group<D>(G, o->eps_tol, nullptr, piB_next, nullptr);
    resid_side<D>(G, 0, piB_next, piB);
    resid_side<D>(G, 1, iS_new, iS_prev);
    if ((s = read_status(G))) return s;
    const double *res = h_res(G);
    std::swap(piB, piB_next);
    std::swap(iS_new, iS_prev);
    double dS2 = 0.0, nS2 = 0.0;
    for (int i = 0; i < n; ++i) {
      dS2 += res[2 * n + 2 * i];
      nS2 += res[2 * n + 2 * i + 1];
    }
    st.r_B = std::sqrt(res[0]) / std::max(std::sqrt(res[1]), 1e-30);
    st.r_S = std::sqrt(dS2) / std::max(std::sqrt(nS2), 1e-30);
    st.iters = k + 1;
    if (st.r_B <= o->eps_conv && st.r_S <= o->eps_conv) {
      st.converged = 1;
      break;
    }
  }
  // the coarse particles move with the last coarse solution
  g2p_side<D, TB>(G, 0, dT);
  count_recv<D>(G);
  if ((s = read_status(G))) return s;
  const int *amb = h_int(G, G->off_amb);
  const int *nrecv = h_int(G, G->off_recv);
  st.n_recv_B = nrecv[0];
  for (int i = 0; i < n; ++i) {
    st.n_amb += amb[i];
    st.n_recv_S += nrecv[n + i];
  }
  if (out) *out = st;
  return OSMPM_OK;
}

template <int D, typename TB>
osmpm_status single_group(osmpm_batch *G, double dt, const osmpm_solve_opts *o, osmpm_solve_stats *out) {
  osmpm_status s;
  if ((s = group_sync(G))) return s;
  std::vector<int> one(G->n, 1);
  set_active(G, 0, one);
  p2g_side<D, TB>(G, 0, false);
  std::vector<osmpm_solve_stats> ss;
  if ((s = solve_side<D, TB>(G, 0, dt, 0, kBufVbc, o, &ss))) return s;
  g2p_side<D, TB>(G, 0, dt);
  if ((s = read_status(G))) return s;
  if (out)
    for (int i = 0; i < G->n; ++i) out[i] = ss[i];
  return OSMPM_OK;
}

// Single-domain entry points work on the domain's group of one.
osmpm_status solo_ready(osmpm_domain *d) {
  osmpm_status s = group_sync(d->solo);
  if (s) return s;
  set_active(d->solo, 0, std::vector<int>(1, 1));
  return OSMPM_OK;
}

template <int D, typename TB>
osmpm_status p2g_solo(osmpm_domain *d) {
  osmpm_status s = solo_ready(d);
  if (s) return s;
  p2g_side<D, TB>(d->solo, 0, true);
  return check_launch(d->ctx);
}

template <int D, typename TB>
osmpm_status solve_solo(osmpm_domain *d, double dt, int use_schwarz, const osmpm_solve_opts *o,
                        osmpm_solve_stats *st) {
  osmpm_status s = solo_ready(d);
  if (s) return s;
  std::vector<osmpm_solve_stats> ss;
  if ((s = solve_side<D, TB>(d->solo, 0, dt, use_schwarz, kBufVbc, o, &ss))) return s;
  if (st) *st = ss[0];
  return OSMPM_OK;
}

template <int D, typename TB>
osmpm_status g2p_solo(osmpm_domain *d, double dt) {
  osmpm_status s = solo_ready(d);
  if (s) return s;
  g2p_side<D, TB>(d->solo, 0, dt);
  return check_launch(d->ctx);
}

// The group of one coarse/fine pair, created on first use and kept by B.
osmpm_status pair_group(osmpm_domain *B, osmpm_domain *S, osmpm_batch **out) {
  if (B->pair && B->pair_uid == S->uid && !B->pair->dead) {
    *out = B->pair;
  } else {
    if (B->pair) group_free(B->pair);
    B->pair = nullptr;
    osmpm_status s = group_create(B->ctx, 1, &B, &S, &B->pair);
    if (s) return s;
    B->pair_uid = S->uid;
    *out = B->pair;
  }
  osmpm_status s = group_sync(*out);
  if (s) return s;
  set_all_active(*out);
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

bool pair_ok(const osmpm_domain *B, const osmpm_domain *S) {
  return B && S && B != S && B->ctx == S->ctx && B->D == S->D && B->desc.h0 == S->desc.h0 && B->m_ref == S->m_ref &&
         B->precision == S->precision;
}

// ---------------------------------------------------------------- reverse mode
// Stored forward state of one domain at one point of a frame: the particle
// arrays in their sorted order (as the kernels of that point saw them), the
// bins, the grid from their P2G, the scene-BC mask and, for a point that
// starts a solve, its solution and Schwarz data.
struct TapePoint {
  std::vector<void *> allocs;
  PartPtrs p{};
  int *cell_start = nullptr;
  double *m = nullptr, *vn = nullptr, *u = nullptr, *vbc = nullptr;
  int8_t *bcg = nullptr;
};

void tape_free(TapePoint &t) {
  for (void *q : t.allocs) (void)hipFree(q);
  t.allocs.clear();
}

// Device memory of one call's work arrays.  By default every request is a
// hipMalloc, freed by release().  With a fixed region (base set), requests
// are carved out of [base, base + cap) at 256-byte alignment, release() frees
// nothing, and a request past cap fails with OSMPM_E_INVALID_ARG.  In
// measuring mode nothing is allocated and `used` sums the aligned sizes (the
// returned pointers are placeholders that must not be dereferenced).
struct Arena {
  osmpm_ctx *c = nullptr;
  char *base = nullptr;
  size_t cap = 0, used = 0;
  bool measure = false;
  std::vector<void *> owned;
  osmpm_status get(size_t bytes, void **p) {
    const size_t nb = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    if (measure) {
      *p = reinterpret_cast<void *>((uintptr_t)256);
      used += nb;
      return OSMPM_OK;
    }
    if (base) {
      if (nb > cap - used)
        return fail(c, OSMPM_E_INVALID_ARG, "work arrays exceed the fixed device region of " + std::to_string(cap) +
                                                " bytes");
      *p = base + used;
      used += nb;
      return OSMPM_OK;
    }
    return dalloc_bytes(c, owned, p, bytes);
  }
  void release() {
    for (void *q : owned) (void)hipFree(q);
    owned.clear();
  }
};

// Work arrays of a tape point, from the arena A (default: hipMalloc'ed into
// t.allocs, freed by tape_free).
osmpm_status tape_alloc(osmpm_domain *d, TapePoint &t, Arena *A = nullptr, bool particles_only = false) {
  osmpm_ctx *c = d->ctx;
  const size_t cap = (size_t)d->cap, nn = (size_t)d->g.nn, nd = nn * d->D;
  const int D = d->D;
  osmpm_status s = OSMPM_OK;
  void *q = nullptr;
  auto al = [&](size_t bytes) -> void * {
    if (s) return nullptr;
    s = A ? A->get(bytes, &q) : dalloc_bytes(c, t.allocs, &q, bytes);
    return s ? nullptr : q;
  };
  t.p.x = (double *)al(cap * D * sizeof(double));
  t.p.v = al(cap * D * d->tb);
  t.p.B = al(cap * D * D * d->tb);
  t.p.F = al(cap * D * D * d->tb);
  t.p.mass = (double *)al(cap * sizeof(double));
  t.p.vol = (double *)al(cap * sizeof(double));
  t.p.mat = (int *)al(cap * sizeof(int));
  t.p.id = (int *)al(cap * sizeof(int));
  t.p.flags = (uint8_t *)al(cap);
  t.cell_start = (int *)al(((size_t)d->nk + 1) * sizeof(int));
  if (particles_only) {
    if (s) tape_free(t);
    return s;
  }
  t.m = (double *)al(nn * sizeof(double));
  t.vn = (double *)al(nd * sizeof(double));
  t.u = (double *)al(nd * sizeof(double));
  t.vbc = (double *)al(nd * sizeof(double));
  t.bcg = (int8_t *)al(nd);
  if (s) tape_free(t);
  return s;
}

// Copies between the domain's current buffers and a tape point; `dir` > 0
// saves, < 0 loads.  what: bit 0 particles and bins, bit 1 grid, bit 2 the
// solution u, bit 3 the Schwarz data.
osmpm_status tape_copy(osmpm_domain *d, TapePoint &t, int dir, int what) {
  osmpm_ctx *c = d->ctx;
  const size_t cap = (size_t)d->cap, nn = (size_t)d->g.nn, nd = nn * d->D;
  const int D = d->D;
  PartPtrs &cp = d->pb[d->cur];
  auto cpy = [&](void *dev, void *tp, size_t bytes) -> hipError_t {
    return dir > 0 ? hipMemcpyAsync(tp, dev, bytes, hipMemcpyDeviceToDevice, c->stream)
                   : hipMemcpyAsync(dev, tp, bytes, hipMemcpyDeviceToDevice, c->stream);
  };
  if (what & 1) {
    HIP_TRY(c, cpy(cp.x, t.p.x, cap * D * sizeof(double)));
    HIP_TRY(c, cpy(cp.v, t.p.v, cap * D * d->tb));
    HIP_TRY(c, cpy(cp.B, t.p.B, cap * D * D * d->tb));
    HIP_TRY(c, cpy(cp.F, t.p.F, cap * D * D * d->tb));
    HIP_TRY(c, cpy(cp.mass, t.p.mass, cap * sizeof(double)));
    HIP_TRY(c, cpy(cp.vol, t.p.vol, cap * sizeof(double)));
    HIP_TRY(c, cpy(cp.mat, t.p.mat, cap * sizeof(int)));
    HIP_TRY(c, cpy(cp.id, t.p.id, cap * sizeof(int)));
    HIP_TRY(c, cpy(cp.flags, t.p.flags, cap));
    HIP_TRY(c, cpy(d->cell_start, t.cell_start, ((size_t)d->nk + 1) * sizeof(int)));
  }
  if (what & 2) {
    HIP_TRY(c, cpy(d->m, t.m, nn * sizeof(double)));
    HIP_TRY(c, cpy(d->vn, t.vn, nd * sizeof(double)));
    HIP_TRY(c, cpy(d->bcg, t.bcg, nd));
  }
  if (what & 4) HIP_TRY(c, cpy(d->u, t.u, nd * sizeof(double)));
  if (what & 8) HIP_TRY(c, cpy(d->vbc, t.vbc, nd * sizeof(double)));
  return OSMPM_OK;
}

// Particle adjoint in particle-id order, component-major [component][np].
struct AdjState {
  double *x = nullptr, *v = nullptr, *B = nullptr, *F = nullptr;
};

template <typename Get>
osmpm_status adj_alloc_with(Get get, int np, int D, AdjState &a) {
  void *q = nullptr;
  const size_t n = (size_t)std::max(np, 1);
  osmpm_status s;
  if ((s = get(n * D * sizeof(double), &q))) return s;
  a.x = (double *)q;
  if ((s = get(n * D * sizeof(double), &q))) return s;
  a.v = (double *)q;
  if ((s = get(n * D * D * sizeof(double), &q))) return s;
  a.B = (double *)q;
  if ((s = get(n * D * D * sizeof(double), &q))) return s;
  a.F = (double *)q;
  return OSMPM_OK;
}

osmpm_status adj_alloc(osmpm_ctx *c, std::vector<void *> &list, int np, int D, AdjState &a) {
  return adj_alloc_with([&](size_t b, void **q) { return dalloc_bytes(c, list, q, b); }, np, D, a);
}

osmpm_status adj_alloc(Arena &A, int np, int D, AdjState &a) {
  return adj_alloc_with([&](size_t b, void **q) { return A.get(b, q); }, np, D, a);
}

osmpm_status adj_zero(osmpm_ctx *c, const AdjState &a, int np, int D) {
  const size_t n = (size_t)std::max(np, 1);
  HIP_TRY(c, hipMemsetAsync(a.x, 0, n * D * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(a.v, 0, n * D * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(a.B, 0, n * D * D * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(a.F, 0, n * D * D * sizeof(double), c->stream));
  return OSMPM_OK;
}

osmpm_status zero_bytes(osmpm_ctx *c, void *p, size_t bytes) {
  HIP_TRY(c, hipMemsetAsync(p, 0, bytes, c->stream));
  return OSMPM_OK;
}

// Caller layout ([n][d], [n][d][d] rows in input order) <-> component-major.
void adj_from_rows(osmpm_ctx *c, int np, int D, const double *x, const double *v, const double *B, const double *F,
                   const AdjState &a) {
  const dim3 gb(blocks_for((int64_t)np * D * D, 2048)), blk(kBlock);
  launch(c, -1, 0, -1, k_aos_to_soa<double>, gb, blk, 0, (int64_t)np, D, x, a.x, (int64_t)np, 0);
  launch(c, -1, 0, -1, k_aos_to_soa<double>, gb, blk, 0, (int64_t)np, D, v, a.v, (int64_t)np, 0);
  launch(c, -1, 0, -1, k_aos_to_soa<double>, gb, blk, 0, (int64_t)np, D * D, B, a.B, (int64_t)np, 0);
  launch(c, -1, 0, -1, k_aos_to_soa<double>, gb, blk, 0, (int64_t)np, D * D, F, a.F, (int64_t)np, 0);
}
void adj_to_rows(osmpm_ctx *c, int np, int D, const AdjState &a, double *x, double *v, double *B, double *F) {
  const dim3 gb(blocks_for((int64_t)np * D * D, 2048)), blk(kBlock);
  launch(c, -1, 0, -1, k_soa_to_aos<double>, gb, blk, 0, (int64_t)np, D, (const double *)a.x, (int64_t)np, x, 0);
  launch(c, -1, 0, -1, k_soa_to_aos<double>, gb, blk, 0, (int64_t)np, D, (const double *)a.v, (int64_t)np, v, 0);
  launch(c, -1, 0, -1, k_soa_to_aos<double>, gb, blk, 0, (int64_t)np, D * D, (const double *)a.B, (int64_t)np, B, 0);
  launch(c, -1, 0, -1, k_soa_to_aos<double>, gb, blk, 0, (int64_t)np, D * D, (const double *)a.F, (int64_t)np, F, 0);
}

// P2G transposed on a stored point of domain d.
template <int D, typename TB>
void adj_p2g(osmpm_domain *d, const TapePoint &t, const double *mbar, const double *vnbar, const AdjState &a) {
  if (d->np == 0) return;
  launch(d->ctx, -1, 0, -1, k_adj_p2g<D, TB>, dim3(blocks_for(d->np)), dim3(kBlock), 0, d->g, d->np, d->cap,
         (const double *)t.p.x, (const TB *)t.p.v, (const TB *)t.p.B, (const double *)t.p.mass, (const int *)t.p.id,
         (const double *)t.m, (const double *)t.vn, mbar, vnbar, a.x, a.v, a.B);
}

// G2P transposed on a stored point (state before G2P, its grid, u).
template <int D, typename TB>
void adj_g2p(osmpm_domain *d, const TapePoint &t, const double *u, double dt, const AdjState &in, double *ubar,
             const AdjState &out) {
  if (d->np == 0) return;
  launch(d->ctx, -1, 0, -1, k_adj_g2p<D, TB>, dim3(blocks_for(d->np)), dim3(kBlock), 0, d->g, d->np, d->cap,
         (const double *)t.p.x, (const TB *)t.p.F, (const int *)t.p.id, (const double *)t.m, u, dt,
         (const double *)in.x, (const double *)in.v, (const double *)in.B, (const double *)in.F, ubar, out.x,
         out.F);
}

// Adjoint of the implicit solve of side s of a group of one, whose current
// buffers hold the stored point (particles, bins, grid, scene-BC mask) and
// whose solution is u_tape.  The tangents are rebuilt at the solution
// without PSD projection, H_ff lambda = ubar_f is solved on the forward CG
// kernels, and the input terms are scattered.
template <int D, typename TB>
osmpm_status adj_solve(osmpm_batch *G, int s, double dt, int use_schwarz, const osmpm_solve_opts *o,
                       double adj_rtol, const double *u_tape, const double *ubar, double *mbar, double *vnbar,
                       double *vbcbar, double *hl, const AdjState &a, double *mubar, double *lambar) {
  osmpm_ctx *c = G->c;
  osmpm_domain *d = G->dom[s][0];
  const Ext &E = G->ext[s];
  const DomDesc *dd = G->dd[s];
  const int n = G->n, nd = d->g.nn * d->D;
  const dim3 blk(kBlock);
  set_active(G, s, std::vector<int>(n, 1));
  // the work lists of the restored binning and grid
  build_tile_list(G, s);
  build_node_list(G, s, false);
  launch(c, -1, 0, -1, k_bc_init<D, TB>, dim3(E.node_blocks, n), blk, 0, dd, dt, use_schwarz, kBufVbc, -1);
  HIP_TRY(c, hipMemcpyAsync(d->u, u_tape, (size_t)nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  launch(c, -1, 0, -1, k_solve_begin, dim3(1, n), blk, 0, dd, dt, -1);
  launch(c, -1, 0, -1, k_grad_hess<D, TB>, dim3(E.tile_blocks, n), blk, E.lds_grad, dd, 0, G->err);
  launch(c, -1, 0, -1, k_grad_node<D, TB>, dim3(E.node_blocks, n), blk, 0, dd, dt, o->gravity[0], o->gravity[1],
         o->gravity[2]);
  launch(c, -1, 0, -1, k_adj_set_rhs, dim3(E.node_blocks, n), blk, 0, dd, ubar);
  launch(c, -1, 0, -1, k_cg_init<D, TB>, dim3(E.node_blocks, n), blk, 0, dd, 0, 0.0, 0.0, 0, 0.0);
  const int max_cg = 20000, chunk = 16;
  osmpm_status st;
  for (int launched = 0;; launched += chunk) {
    for (int j = 0; j < chunk; ++j)
      launch(c, -1, 0, -1, k_cg_iter<D, TB>, dim3(E.tile_blocks, n), blk, E.lds_hvp, dd, j & 1, dt, adj_rtol,
             max_cg, 0);
    if ((st = read_status(G))) return st;
    if (h_cg(G, s)[0].done) break;
    if (launched > max_cg + chunk) return fail(c, OSMPM_E_STATE, "adjoint CG did not terminate");
  }
  if ((st = zero_bytes(c, hl, (size_t)nd * sizeof(double)))) return st;
  if (d->np > 0)
    launch(c, -1, 0, -1, k_adj_hvp<D, TB>, dim3(blocks_for(d->np), n), blk, 0, dd, (const TB *)d->del, hl);
  launch(c, -1, 0, -1, k_adj_solve_nodes<D, TB>, dim3(blocks_for(d->g.nn), n), blk, 0, dd, dt, o->gravity[0],
         o->gravity[1], o->gravity[2], ubar, (const double *)hl, use_schwarz, mbar, vnbar, vbcbar);
  if (d->np > 0)
    launch(c, -1, 0, -1, k_adj_solve_particles<D, TB>, dim3(blocks_for(d->np), n), blk, 0, dd, a.x, a.F, d->np,
           mubar, lambar);
  return check_launch(c);
}

// Work arrays of the single-frame adjoint of d: two tape points (the frame's
// start and end), the particle adjoints entering and leaving, the node
// adjoints ubar, vnbar, the product H lambda, the mass adjoint and the
// material sums (64 mu + 64 lambda entries).
struct SingleAdjBufs {
  TapePoint t0, te;
  AdjState ain, aout;
  double *ubar = nullptr, *mbar = nullptr, *vnbar = nullptr, *hl = nullptr, *mat = nullptr;
};

osmpm_status single_adjoint_buffers(osmpm_domain *d, Arena &A, SingleAdjBufs &b) {
  const size_t nn = (size_t)d->g.nn, nd = nn * d->D;
  osmpm_status s;
  void *q = nullptr;
  if ((s = tape_alloc(d, b.t0, &A)) || (s = tape_alloc(d, b.te, &A)) || (s = adj_alloc(A, d->np, d->D, b.ain)) ||
      (s = adj_alloc(A, d->np, d->D, b.aout)))
    return s;
  for (double **pp : {&b.ubar, &b.vnbar, &b.hl}) {
    if ((s = A.get(nd * sizeof(double), &q))) return s;
    *pp = (double *)q;
  }
  if ((s = A.get(nn * sizeof(double), &q))) return s;
  b.mbar = (double *)q;
  if ((s = A.get(128 * sizeof(double), &q))) return s;
  b.mat = (double *)q;
  return OSMPM_OK;
}

// Bytes the single-frame adjoint of d takes from a fixed region.
size_t single_adjoint_bytes(osmpm_domain *d) {
  Arena A;
  A.c = d->ctx;
  A.measure = true;
  SingleAdjBufs b;
  (void)single_adjoint_buffers(d, A, b);
  return A.used;
}

// Adjoint of one single-domain frame (P2G, solve, G2P) of d; see the ABI.
// Work arrays come from the arena A: hipMalloc'ed for this call, or carved
// out of a fixed device region (every one of them is written before it is
// read, so the region's previous contents do not matter).
template <int D, typename TB>
osmpm_status single_adjoint_impl(osmpm_domain *d, double dt, const osmpm_solve_opts *o, double adj_rtol,
                                 const double *const *in, double *const *out, double *mubar_h, double *lambar_h,
                                 Arena &A) {
  osmpm_ctx *c = d->ctx;
  osmpm_batch *G = d->solo;
  osmpm_status s;
  if ((s = group_sync(G))) return s;
  set_active(G, 0, std::vector<int>(1, 1));
  const int np = d->np, nn = d->g.nn, nd = nn * D;
  SingleAdjBufs bufs;
  TapePoint &t0 = bufs.t0, &te = bufs.te;
  const AdjState &ain = bufs.ain, &aout = bufs.aout;
  auto cleanup = [&]() {
    tape_free(t0);
    tape_free(te);
    A.release();
  };
  if ((s = single_adjoint_buffers(d, A, bufs))) {
    cleanup();
    return s;
  }
  double *ubar = bufs.ubar, *mbar = bufs.mbar, *vnbar = bufs.vnbar, *hl = bufs.hl, *mat = bufs.mat;
  // forward with storage
  p2g_side<D, TB>(G, 0, false);
  if ((s = tape_copy(d, t0, 1, 1 | 2))) return cleanup(), s;
  std::vector<osmpm_solve_stats> ss;
  if ((s = solve_side<D, TB>(G, 0, dt, 0, kBufVbc, o, &ss))) return cleanup(), s;
  if ((s = tape_copy(d, t0, 1, 4))) return cleanup(), s;
  g2p_side<D, TB>(G, 0, dt);
  if ((s = tape_copy(d, te, 1, 1 | 2 | 4))) return cleanup(), s;
  // reverse
  adj_from_rows(c, np, D, in[0], in[1], in[2], in[3], ain);
  if ((s = adj_zero(c, aout, np, D)) || (s = zero_bytes(c, ubar, (size_t)nd * 8)) ||
      (s = zero_bytes(c, mbar, (size_t)nn * 8)) || (s = zero_bytes(c, vnbar, (size_t)nd * 8)) ||
      (s = zero_bytes(c, mat, 128 * 8)))
    return cleanup(), s;
  adj_g2p<D, TB>(d, t0, t0.u, dt, ain, ubar, aout);
  if ((s = tape_copy(d, t0, -1, 1 | 2))) return cleanup(), s;
  if ((s = adj_solve<D, TB>(G, 0, dt, 0, o, adj_rtol, t0.u, ubar, mbar, vnbar, nullptr, hl, aout, mat, mat + 64)))
    return cleanup(), s;
  adj_p2g<D, TB>(d, t0, mbar, vnbar, aout);
  if ((s = tape_copy(d, te, -1, 1 | 2 | 4))) return cleanup(), s;
  adj_to_rows(c, np, D, aout, out[0], out[1], out[2], out[3]);
  // the material sums come back through the context's pinned staging
  // buffer (at least 64 KB from creation)
  const double *hm = reinterpret_cast<const double *>(c->h_pin);
  HIP_TRY(c, hipMemcpyAsync(c->h_pin, mat, 128 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if ((s = read_status(G))) return cleanup(), s;
  for (int k = 0; k < d->n_mat; ++k) {
    mubar_h[k] += hm[k];
    lambar_h[k] += hm[64 + k];
  }
  cleanup();
  return OSMPM_OK;
}

// Adjoint of one Schwarz frame of the pair (B, S) with exactly K Schwarz
// iterations (the forward's count): the frame is recomputed with storage and
// swept in reverse in the order of the oracle's reverse mode; see the ABI.
template <int D, typename TB>
osmpm_status schwarz_adjoint_impl(osmpm_batch *G, double dT, const osmpm_schwarz_opts *o, int K, double adj_rtol,
                                  int implicit, double fp_tol, int fp_max, int *fp_used,
                                  const double *const *inB, const double *const *inS, double *const *outB,
                                  double *const *outS, double *mat_h) {
  osmpm_ctx *c = G->c;
  osmpm_domain *B = G->dom[0][0], *S = G->dom[1][0];
  const int M = o->M;
  const double dt = dT / (double)M;
  const int npB = B->np, npS = S->np, nnB = B->g.nn, nnS = S->g.nn, ndB = nnB * D, ndS = nnS * D;
  osmpm_status s;
  if ((s = group_sync(G))) return s;
  // Stored iterations: all K (unrolled) or only the last (implicit: every
  // adjoint pass is linearised there); iteration k lives in slot sl(k).
  const int n_slots = implicit ? 1 : K;
  auto sl = [&](int k) -> size_t { return implicit ? 0 : (size_t)k; };
  std::vector<void *> mem;
  TapePoint tB0, tBe;
  std::vector<TapePoint> tS((size_t)n_slots * (M + 1));
  auto cleanup = [&]() {
    tape_free(tB0);
    tape_free(tBe);
    for (TapePoint &t : tS) tape_free(t);
    for (void *q : mem) (void)hipFree(q);
  };
  void *q = nullptr;
  auto dbl = [&](size_t n, double **pp) -> osmpm_status {
    osmpm_status r = dalloc_bytes(c, mem, &q, std::max<size_t>(n, 1) * sizeof(double));
    if (!r) *pp = (double *)q;
    return r;
  };
  double *uB = nullptr, *piB = nullptr, *ubarB = nullptr, *ubarBk = nullptr, *mbarB = nullptr, *vnbarB = nullptr,
         *vBkbar = nullptr, *pibar = nullptr, *pibar_next = nullptr, *hlB = nullptr, *ubarS = nullptr,
         *mbarS = nullptr, *vnbarS = nullptr, *vbcbar = nullptr, *gSn = nullptr, *gSn1 = nullptr, *hlS = nullptr,
         *mat = nullptr, *nrm = nullptr;
  AdjState aBin, aBo, aSin, aS, aP, aS0;
  if ((s = tape_alloc(B, tB0)) || (s = tape_alloc(B, tBe)) || (s = dbl((size_t)n_slots * ndB, &uB)) ||
      (s = dbl((size_t)n_slots * ndB, &piB)) || (s = dbl(ndB, &ubarB)) || (s = dbl(ndB, &ubarBk)) ||
      (s = dbl(nnB, &mbarB)) || (s = dbl(ndB, &vnbarB)) || (s = dbl(ndB, &vBkbar)) || (s = dbl(ndB, &pibar)) ||
      (s = dbl(ndB, &pibar_next)) || (s = dbl(ndB, &hlB)) || (s = dbl(ndS, &ubarS)) || (s = dbl(nnS, &mbarS)) ||
      (s = dbl(ndS, &vnbarS)) || (s = dbl(ndS, &vbcbar)) || (s = dbl(ndS, &gSn)) || (s = dbl(ndS, &gSn1)) ||
      (s = dbl(ndS, &hlS)) || (s = dbl(256, &mat)) || (s = dbl(1, &nrm)) || (s = adj_alloc(c, mem, npB, D, aBin)) ||
      (s = adj_alloc(c, mem, npB, D, aBo)) || (s = adj_alloc(c, mem, npS, D, aSin)) ||
      (s = adj_alloc(c, mem, npS, D, aS)) || (s = adj_alloc(c, mem, npS, D, aP)) ||
      (s = adj_alloc(c, mem, npS, D, aS0))) {
    cleanup();
    return s;
  }
  for (TapePoint &t : tS)
    if ((s = tape_alloc(S, t))) return cleanup(), s;
  const DomDesc *ddB = G->dd[0], *ddS = G->dd[1];
  const dim3 blk(kBlock);

  // ---- forward recompute with storage
  set_all_active(G);
  copy_state_side<D, TB>(G, 1, 1);
  p2g_side<D, TB>(G, 0, true);
  p2g_side<D, TB>(G, 1, true);
  if ((s = tape_copy(B, tB0, 1, 1 | 2))) return cleanup(), s;
  interface_group<D>(G);
  project_group<D>(G, o->eps_tol, nullptr, 0, nullptr);
  HIP_TRY(c, hipMemcpyAsync(piB, B->w0, (size_t)ndB * 8, hipMemcpyDeviceToDevice, c->stream));
  for (int k = 0; k < K; ++k) {
    HIP_TRY(c, hipMemcpyAsync(B->w0, piB + sl(k) * ndB, (size_t)ndB * 8, hipMemcpyDeviceToDevice, c->stream));
    if ((s = solve_side<D, TB>(G, 0, dT, 1, 0, &o->coarse, nullptr))) return cleanup(), s;
    HIP_TRY(c, hipMemcpyAsync(uB + sl(k) * ndB, B->u, (size_t)ndB * 8, hipMemcpyDeviceToDevice, c->stream));
    launch(c, -1, 0, -1, k_vel_from_u<D>, dim3(blocks_for(nnB), 1), blk, 0, ddB, dT);
    copy_state_side<D, TB>(G, 1, 0);
    p2g_side<D, TB>(G, 1, false);
    TapePoint &t0 = tS[sl(k) * (M + 1)];
    if ((s = tape_copy(S, t0, 1, 1 | 2))) return cleanup(), s;
    interp_group<D>(G, kBufVn, nullptr, 0, nullptr);
    interp_group<D>(G, 2, nullptr, 1, nullptr);
    for (int m = 1; m <= M; ++m) {
      TapePoint &tp = tS[sl(k) * (M + 1) + (m - 1)];
      launch(c, -1, 0, -1, k_temporal<D>, dim3(blocks_for(ndS, 1024), 1), blk, 0, ddS, (double)m / (double)M, 0, 1);
      if ((s = tape_copy(S, tp, 1, 8))) return cleanup(), s;
      if ((s = solve_side<D, TB>(G, 1, dt, 1, kBufVbc, &o->fine, nullptr))) return cleanup(), s;
      if ((s = tape_copy(S, tp, 1, 4))) return cleanup(), s;
      g2p_side<D, TB>(G, 1, dt);
      p2g_side<D, TB>(G, 1, false);
      if ((s = tape_copy(S, tS[sl(k) * (M + 1) + m], 1, 1 | 2))) return cleanup(), s;
    }
    if (k + 1 < K) {
      project_group<D>(G, o->eps_tol, nullptr, 0, nullptr);
      HIP_TRY(c, hipMemcpyAsync(piB + sl(k + 1) * ndB, B->w0, (size_t)ndB * 8, hipMemcpyDeviceToDevice,
                                c->stream));
    }
  }
  HIP_TRY(c, hipMemcpyAsync(B->u, uB + sl(K - 1) * ndB, (size_t)ndB * 8, hipMemcpyDeviceToDevice, c->stream));
  g2p_side<D, TB>(G, 0, dT);
  if ((s = tape_copy(B, tBe, 1, 1 | 2 | 4))) return cleanup(), s;
  if ((s = read_status(G))) return cleanup(), s;

  // ---- reverse sweep (adjoints in particle-id order)
  adj_from_rows(c, npB, D, inB[0], inB[1], inB[2], inB[3], aBin);
  adj_from_rows(c, npS, D, inS[0], inS[1], inS[2], inS[3], aSin);
  if ((s = adj_zero(c, aBo, npB, D)) || (s = adj_zero(c, aS0, npS, D)) || (s = zero_bytes(c, ubarB, ndB * 8)) ||
      (s = zero_bytes(c, mbarB, nnB * 8)) || (s = zero_bytes(c, vnbarB, ndB * 8)) ||
      (s = zero_bytes(c, pibar_next, ndB * 8)) || (s = zero_bytes(c, mat, 256 * 8)))
    return cleanup(), s;
  adj_g2p<D, TB>(B, tB0, uB + sl(K - 1) * ndB, dT, aBin, ubarB, aBo);
  const int64_t nsS = (int64_t)npS * (2 * D + 2 * D * D);
  double w_norm = 0.0;
  for (int j = 0;; ++j) {
    // unrolled: iteration k = K-1-j; implicit: pass j of the Neumann series
    // of the fixed-point adjoint, always on the last iteration
    const int k = implicit ? K - 1 : K - 1 - j;
    if (k < 0) break;
    if (j == 0) {
      HIP_TRY(c, hipMemcpyAsync(ubarBk, ubarB, (size_t)ndB * 8, hipMemcpyDeviceToDevice, c->stream));
      for (int f = 0; f < 4; ++f) {
        const size_t bytes = (size_t)std::max(npS, 1) * (f < 2 ? D : D * D) * 8;
        const double *src = f == 0 ? aSin.x : f == 1 ? aSin.v : f == 2 ? aSin.B : aSin.F;
        double *dst = f == 0 ? aS.x : f == 1 ? aS.v : f == 2 ? aS.B : aS.F;
        HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
      }
    } else {
      if ((s = zero_bytes(c, ubarBk, ndB * 8)) || (s = adj_zero(c, aS, npS, D))) return cleanup(), s;
      // the projection of the grid after the last sub-step fed coarse solve k+1
      TapePoint &tl = tS[sl(k) * (M + 1) + M];
      if ((s = tape_copy(S, tl, -1, 2))) return cleanup(), s;
      launch(c, -1, 0, -1, k_zero_proj, dim3(blocks_for(ndB, 1024), 1), blk, 0, ddB);
      launch(c, -1, 0, -1, k_project_scatter<D>, dim3(blocks_for(nnS), 1), blk, 0, ddS, ddB, (const double *)nullptr,
             G->err);
      if ((s = zero_bytes(c, mbarS, nnS * 8)) || (s = zero_bytes(c, vnbarS, ndS * 8))) return cleanup(), s;
      launch(c, -1, 0, -1, k_adj_project<D>, dim3(blocks_for(nnS)), blk, 0, B->g, S->g, (const double *)tl.m,
             (const double *)tl.vn, (const uint8_t *)B->recv, (const double *)B->pnum, (const double *)B->pden,
             o->eps_tol, (const double *)pibar_next, mbarS, vnbarS);
      adj_p2g<D, TB>(S, tl, mbarS, vnbarS, aS);
    }
    if ((s = zero_bytes(c, gSn, ndS * 8)) || (s = zero_bytes(c, gSn1, ndS * 8))) return cleanup(), s;
    for (int m = M; m >= 1; --m) {
      TapePoint &tp = tS[sl(k) * (M + 1) + (m - 1)];
      if ((s = adj_zero(c, aP, npS, D)) || (s = zero_bytes(c, ubarS, ndS * 8))) return cleanup(), s;
      adj_g2p<D, TB>(S, tp, tp.u, dt, aS, ubarS, aP);
      if ((s = tape_copy(S, tp, -1, 1 | 2 | 8))) return cleanup(), s;
      if ((s = zero_bytes(c, mbarS, nnS * 8)) || (s = zero_bytes(c, vnbarS, ndS * 8)) ||
          (s = zero_bytes(c, vbcbar, ndS * 8)))
        return cleanup(), s;
      if ((s = adj_solve<D, TB>(G, 1, dt, 1, &o->fine, adj_rtol, tp.u, ubarS, mbarS, vnbarS, vbcbar, hlS, aP,
                                mat + 128, mat + 192)))
        return cleanup(), s;
      launch(c, -1, 0, -1, k_adj_temporal, dim3(blocks_for(ndS, 1024)), blk, 0, (int64_t)ndS, (double)m / (double)M,
             (const double *)vbcbar, gSn, gSn1);
      adj_p2g<D, TB>(S, tp, mbarS, vnbarS, aP);
      std::swap(aS, aP);
    }
    // restore of the stored fine state
    launch(c, -1, 0, -1, k_axpy_d, dim3(blocks_for(nsS, 2048)), blk, 0, (int64_t)npS * D, 1.0, (const double *)aS.x,
           aS0.x);
    launch(c, -1, 0, -1, k_axpy_d, dim3(blocks_for(nsS, 2048)), blk, 0, (int64_t)npS * D, 1.0, (const double *)aS.v,
           aS0.v);
    launch(c, -1, 0, -1, k_axpy_d, dim3(blocks_for(nsS, 2048)), blk, 0, (int64_t)npS * D * D, 1.0,
           (const double *)aS.B, aS0.B);
    launch(c, -1, 0, -1, k_axpy_d, dim3(blocks_for(nsS, 2048)), blk, 0, (int64_t)npS * D * D, 1.0,
           (const double *)aS.F, aS0.F);
    // interpolations I(v_B^(k+1)) and I(v_B^n)
    if ((s = zero_bytes(c, vBkbar, ndB * 8))) return cleanup(), s;
    launch(c, -1, 0, -1, k_adj_interp<D>, dim3(blocks_for(nnS)), blk, 0, B->g, S->g, (const double *)tB0.m,
           (const uint8_t *)S->recv, (const double *)gSn1, vBkbar);
    launch(c, -1, 0, -1, k_adj_interp<D>, dim3(blocks_for(nnS)), blk, 0, B->g, S->g, (const double *)tB0.m,
           (const uint8_t *)S->recv, (const double *)gSn, vnbarB);
    launch(c, -1, 0, -1, k_adj_vel<D>, dim3(blocks_for(nnB)), blk, 0, nnB, (const double *)tB0.m,
           (const double *)vBkbar, dT, ubarBk);
    // coarse solve k
    if ((s = tape_copy(B, tB0, -1, 1 | 2))) return cleanup(), s;
    HIP_TRY(c, hipMemcpyAsync(B->vbc, piB + sl(k) * ndB, (size_t)ndB * 8, hipMemcpyDeviceToDevice, c->stream));
    if ((s = zero_bytes(c, pibar, ndB * 8))) return cleanup(), s;
    if ((s = adj_solve<D, TB>(G, 0, dT, 1, &o->coarse, adj_rtol, uB + sl(k) * ndB, ubarBk, mbarB, vnbarB, pibar,
                              hlB, aBo, mat, mat + 64)))
      return cleanup(), s;
    HIP_TRY(c, hipMemcpyAsync(pibar_next, pibar, (size_t)ndB * 8, hipMemcpyDeviceToDevice, c->stream));
    if (implicit) {
      // pibar = (Phi_z^T)^j w, w = pibar of pass 0
      launch(c, -1, 0, -1, k_sumsq_d, dim3(1), blk, 0, (int64_t)ndB, (const double *)pibar, nrm);
      double h = 0.0;
      HIP_TRY(c, hipMemcpyAsync(&h, nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      h = std::sqrt(h);
      if (j == 0) w_norm = h;
      *fp_used = j;
      if (fp_tol > 0.0 && h <= fp_tol * w_norm) break;
      if (j == fp_max) {
        if (fp_tol > 0.0) {
          cleanup();
          return fail(c, OSMPM_E_NOT_CONVERGED, "adjoint Schwarz iteration did not reach fp_tol within fp_max passes");
        }
        break;
      }
    }
  }
  // Step 0: projection of the fine start grid (the first iterate's data, on
  // which the fixed point does not depend), then both P2Gs
  if (!implicit) {
    TapePoint &t00 = tS[0];
    if ((s = tape_copy(S, t00, -1, 2))) return cleanup(), s;
    launch(c, -1, 0, -1, k_zero_proj, dim3(blocks_for(ndB, 1024), 1), blk, 0, ddB);
    launch(c, -1, 0, -1, k_project_scatter<D>, dim3(blocks_for(nnS), 1), blk, 0, ddS, ddB, (const double *)nullptr,
           G->err);
    if ((s = zero_bytes(c, mbarS, nnS * 8)) || (s = zero_bytes(c, vnbarS, ndS * 8))) return cleanup(), s;
    launch(c, -1, 0, -1, k_adj_project<D>, dim3(blocks_for(nnS)), blk, 0, B->g, S->g, (const double *)t00.m,
           (const double *)t00.vn, (const uint8_t *)B->recv, (const double *)B->pnum, (const double *)B->pden,
           o->eps_tol, (const double *)pibar_next, mbarS, vnbarS);
    adj_p2g<D, TB>(S, t00, mbarS, vnbarS, aS0);
  }
  adj_p2g<D, TB>(B, tB0, mbarB, vnbarB, aBo);
  // the pair back at its end-of-frame state
  if ((s = tape_copy(B, tBe, -1, 1 | 2 | 4))) return cleanup(), s;
  if ((s = tape_copy(S, tS[sl(K - 1) * (M + 1) + M], -1, 1 | 2))) return cleanup(), s;
  adj_to_rows(c, npB, D, aBo, outB[0], outB[1], outB[2], outB[3]);
  adj_to_rows(c, npS, D, aS0, outS[0], outS[1], outS[2], outS[3]);
  HIP_TRY(c, hipMemcpyAsync(mat_h, mat, 256 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  s = read_status(G);
  cleanup();
  return s;
}

// ---------------------------------------------------------------- multi-frame runs and their reverse mode
// What a multi-frame run of a Schwarz batch keeps for its reverse mode: the
// run's settings, the scene-BC parameters of every frame (when given), every
// pair's Schwarz iteration count per frame, and the particle state of every
// domain (index side * n + pair) at the start of frames 0, c, 2c, ... (c the
// checkpoint interval) and at the end of the run.  `starts` holds one
// segment's frame start states during the reverse pass.
struct RunRecord {
  int n_frames = 0, every = 1;
  double dT = 0.0;
  osmpm_schwarz_opts o{};
  std::vector<double> bc;  // [n_frames][n][2][kMaxGroups][8]; empty: parameters left as they are
  std::vector<int> iters;  // [n_frames][n]
  std::vector<std::vector<TapePoint>> ckpt;
  std::vector<TapePoint> end;
  std::vector<std::vector<TapePoint>> starts;
};

void run_free(RunRecord *r) {
  if (!r) return;
  for (auto &v : r->ckpt)
    for (TapePoint &t : v) tape_free(t);
  for (auto &v : r->starts)
    for (TapePoint &t : v) tape_free(t);
  for (TapePoint &t : r->end) tape_free(t);
  delete r;
}

// Saves (dir > 0) or restores (dir < 0) the particle state of every domain
// of a Schwarz batch; the points are allocated on the first save.
osmpm_status batch_states(osmpm_batch *G, std::vector<TapePoint> &pts, int dir) {
  const int n = G->n;
  osmpm_status s;
  if (pts.empty()) {
    if (dir < 0) return fail(G->c, OSMPM_E_STATE, "no stored state to restore");
    pts.resize((size_t)2 * n);
    for (int sd = 0; sd < 2; ++sd)
      for (int i = 0; i < n; ++i)
        if ((s = tape_alloc(G->dom[sd][i], pts[(size_t)sd * n + i], nullptr, true))) return s;
  }
  for (int sd = 0; sd < 2; ++sd)
    for (int i = 0; i < n; ++i)
      if ((s = tape_copy(G->dom[sd][i], pts[(size_t)sd * n + i], dir, 1))) return s;
  return OSMPM_OK;
}

// Scene-BC parameters of frame f on every domain of the batch (a domain
// whose parameters change gets its descriptor uploaded by the next frame).
void apply_frame_bc(osmpm_batch *G, const RunRecord &R, int f) {
  if (R.bc.empty()) return;
  const int n = G->n;
  for (int i = 0; i < n; ++i)
    for (int sd = 0; sd < 2; ++sd) {
      osmpm_domain *d = G->dom[sd][i];
      const double *p = &R.bc[((((size_t)f * n + i) * 2 + sd) * kMaxGroups) * 8];
      SceneBC bc = d->bc;
      for (int g = 0; g < bc.n_groups; ++g)
        for (int k = 0; k < 8; ++k) bc.param[g][k] = p[g * 8 + k];
      if (std::memcmp(&bc, &d->bc, sizeof(SceneBC)) != 0) {
        d->bc = bc;
        d->version += 1;
      }
    }
}

// n_frames frames of Alg. 1 on every pair of the batch, recording what the
// reverse pass needs (RunRecord); see the ABI.
template <int D, typename TB>
osmpm_status batch_run_impl(osmpm_batch *G, int n_frames, double dT, const osmpm_schwarz_opts *o, int every,
                            const double *bc_host, osmpm_schwarz_stats *stats) {
  const int n = G->n;
  run_free(G->run);
  G->run = nullptr;
  auto *R = new RunRecord();
  R->n_frames = n_frames;
  R->every = every;
  R->dT = dT;
  R->o = *o;
  if (bc_host) R->bc.assign(bc_host, bc_host + (size_t)n_frames * n * 2 * kMaxGroups * 8);
  R->iters.assign((size_t)n_frames * n, 0);
  R->ckpt.resize((size_t)(n_frames + every - 1) / every);
  std::vector<osmpm_schwarz_stats> st(n);
  osmpm_status s = OSMPM_OK;
  for (int f = 0; f < n_frames && !s; ++f) {
    if (f % every == 0 && (s = batch_states(G, R->ckpt[f / every], 1))) break;
    apply_frame_bc(G, *R, f);
    if ((s = schwarz_group<D, TB>(G, dT, o, st.data()))) break;
    for (int i = 0; i < n; ++i) {
      R->iters[(size_t)f * n + i] = st[i].iters;
      if (stats) stats[(size_t)f * n + i] = st[i];
    }
  }
  if (!s) s = batch_states(G, R->end, 1);
  if (!s) s = check_launch(G->c);
  if (s) {
    run_free(R);
    return s;
  }
  G->run = R;
  return OSMPM_OK;
}

// Reverse mode over the last run of the batch; see the ABI.  Each segment of
// `every` frames is restored from its checkpoint and rerun (batched) to
// recover its frame start states; the frames are then swept last to first,
// every pair through its frame adjoint (the unrolled or the implicit one)
// with its recorded iteration count, carrying the particle adjoints and
// summing the Lame-parameter derivatives, which are finally mapped to
// Young's moduli with dmu/dE = 1 / (2 (1 + nu)), dlam/dE = nu / ((1 + nu)
// (1 - 2 nu)).  The domains are left at the end-of-run state.
template <int D, typename TB>
osmpm_status batch_backward_impl(osmpm_batch *G, const double *const *xbB, const double *const *xbS,
                                 double adj_rtol, int implicit, double fp_tol, int fp_max, double *dE_host) {
  osmpm_ctx *c = G->c;
  RunRecord &R = *G->run;
  const int n = G->n;
  std::vector<void *> mem;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(c->stream);
    for (void *q : mem) (void)hipFree(q);
  };
  // adjoint rows [np][d], [np][d][d] of every domain: current and next
  std::vector<std::array<double *, 4>> cur((size_t)2 * n), nxt((size_t)2 * n);
  osmpm_status s;
  for (int sd = 0; sd < 2; ++sd)
    for (int i = 0; i < n; ++i) {
      const osmpm_domain *d = G->dom[sd][i];
      const size_t np = (size_t)std::max(d->np, 1);
      for (auto *v : {&cur, &nxt})
        for (int f = 0; f < 4; ++f) {
          void *q = nullptr;
          const size_t bytes = np * (f < 2 ? D : D * D) * sizeof(double);
          if ((s = dalloc_bytes(c, mem, &q, bytes)) || (s = zero_bytes(c, q, bytes))) return cleanup(), s;
          (*v)[(size_t)sd * n + i][f] = (double *)q;
        }
      const double *xb = sd == 0 ? (xbB ? xbB[i] : nullptr) : (xbS ? xbS[i] : nullptr);
      if (xb && d->np > 0)
        HIP_TRY(c, hipMemcpyAsync(cur[(size_t)sd * n + i][0], xb, (size_t)d->np * D * sizeof(double),
                                  hipMemcpyDeviceToDevice, c->stream));
    }
  std::vector<double> lame((size_t)n * 256, 0.0);  // per pair: mu_B, lam_B, mu_S, lam_S (64 each)
  if (R.starts.size() < (size_t)R.every) R.starts.resize((size_t)R.every);
  for (int sg = (int)R.ckpt.size() - 1; sg >= 0; --sg) {
    const int f0 = sg * R.every, f1 = std::min(f0 + R.every, R.n_frames);
    if ((s = batch_states(G, R.ckpt[(size_t)sg], -1))) return cleanup(), s;
    for (int f = f0; f < f1; ++f) {
      if ((s = batch_states(G, R.starts[(size_t)(f - f0)], 1))) return cleanup(), s;
      if (f + 1 < f1) {
        apply_frame_bc(G, R, f);
        if ((s = schwarz_group<D, TB>(G, R.dT, &R.o, nullptr))) return cleanup(), s;
      }
    }
    for (int f = f1 - 1; f >= f0; --f) {
      if ((s = batch_states(G, R.starts[(size_t)(f - f0)], -1))) return cleanup(), s;
      apply_frame_bc(G, R, f);
      for (int i = 0; i < n; ++i) {
        osmpm_batch *P = nullptr;
        if ((s = pair_group(G->dom[0][i], G->dom[1][i], &P))) return cleanup(), s;
        const size_t kB = (size_t)i, kS = (size_t)n + i;
        const double *inB[4] = {cur[kB][0], cur[kB][1], cur[kB][2], cur[kB][3]};
        const double *inS[4] = {cur[kS][0], cur[kS][1], cur[kS][2], cur[kS][3]};
        double *outB[4] = {nxt[kB][0], nxt[kB][1], nxt[kB][2], nxt[kB][3]};
        double *outS[4] = {nxt[kS][0], nxt[kS][1], nxt[kS][2], nxt[kS][3]};
        double mh[256];
        int used = 0;
        if ((s = schwarz_adjoint_impl<D, TB>(P, R.dT, &R.o, R.iters[(size_t)f * n + i], adj_rtol, implicit, fp_tol,
                                             fp_max, &used, inB, inS, outB, outS, mh)))
          return cleanup(), s;
        for (int k = 0; k < 256; ++k) lame[(size_t)i * 256 + k] += mh[k];
        std::swap(cur[kB], nxt[kB]);
        std::swap(cur[kS], nxt[kS]);
      }
    }
  }
  if ((s = batch_states(G, R.end, -1))) return cleanup(), s;
  size_t off = 0;
  for (int i = 0; i < n; ++i)
    for (int sd = 0; sd < 2; ++sd) {
      const osmpm_domain *d = G->dom[sd][i];
      for (int k = 0; k < d->n_mat; ++k) {
        const double nu = d->nu_h[k];
        const double dmu = 1.0 / (2.0 * (1.0 + nu)), dlam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        dE_host[off++] = lame[(size_t)i * 256 + sd * 128 + k] * dmu + lame[(size_t)i * 256 + sd * 128 + 64 + k] * dlam;
      }
    }
  s = check_launch(c);
  cleanup();
  return s;
}

// ---------------------------------------------------------------- fixed work region
// The device region of osmpm_single_frame_adjoint_noalloc, the entry point
// that allocates nothing: one copy per device, held until the process ends.
// Host code never passes the array's name as an address (in host code it
// only stands for the symbol): its device address on each device is looked
// up once, with that device current, when the first context on the device
// is created, and kept in fixed_region_ptr.
constexpr int kMaxDevices = 64;
std::mutex fixed_region_mu;
void *fixed_region_ptr[kMaxDevices] = {};

// Looks up the region's address on `device` (the current device) once.
int fixed_region_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return 1;
  std::lock_guard<std::mutex> lock(fixed_region_mu);
  if (fixed_region_ptr[device]) return 0;
  void *ptr = nullptr;
  if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return 1;
  fixed_region_ptr[device] = ptr;
  return 0;
}

void *fixed_region(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(fixed_region_mu);
  return fixed_region_ptr[device];
}

}  // namespace

// ====================================================================== ABI
#define DISPATCH(dim, call) ((dim) == 2 ? call<2> : call<3>)
// Dispatch on dimension and bulk type.
#define DISPATCH2(D_, prec_, call) \
  ((D_) == 2 ? ((prec_) == OSMPM_MIXED ? call<2, float> : call<2, double>) \
             : ((prec_) == OSMPM_MIXED ? call<3, float> : call<3, double>))

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
  if (ensure_pin(c, 1 << 16)) {
    delete c;
    return OSMPM_E_NO_MEMORY;
  }
  if (fixed_region_setup(device)) {
    (void)hipHostFree(c->h_pin);
    delete c;
    return OSMPM_E_DEVICE;
  }
  *out = c;
  return OSMPM_OK;
}

osmpm_status osmpm_ctx_set_graphs(osmpm_ctx *ctx, int32_t enable) {
  if (!ctx || enable < 0 || enable > 2) return OSMPM_E_INVALID_ARG;
  ctx->graphs = enable;
  return OSMPM_OK;
}

osmpm_status osmpm_ctx_set_cg_split(osmpm_ctx *ctx, int32_t mode) {
  if (!ctx || mode < -1 || mode > 1) return OSMPM_E_INVALID_ARG;
  ctx->cg_split = mode;
  return OSMPM_OK;
}

osmpm_status osmpm_ctx_set_stream(osmpm_ctx *ctx, void *stream) {
  if (!ctx) return OSMPM_E_INVALID_ARG;
  ctx->stream = (hipStream_t)stream;
  return OSMPM_OK;
}

osmpm_status osmpm_sync(osmpm_ctx *ctx) {
  if (!ctx) return OSMPM_E_INVALID_ARG;
  osmpm_status s = check_launch(ctx);
  if (s) return s;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  prof_harvest(ctx);
  int err = 0;
  for (osmpm_batch *G : ctx->groups) {
    int e = 0;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->h_pin, G->err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(&e, ctx->h_pin, sizeof(int));
    err |= e;
  }
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
  prof_harvest(ctx);
  while (!ctx->groups.empty()) group_free(ctx->groups.back());
  if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
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
  if (!(grid->h0 > 0.0) || grid->dx_q <= 0 || capacity < 0 || capacity > kMaxItems)
    return fail(ctx, OSMPM_E_INVALID_ARG, "bad grid spacing or capacity");
  if ((int64_t)grid->n_nodes[0] * grid->n_nodes[1] * grid->n_nodes[2] > kMaxItems)
    return fail(ctx, OSMPM_E_INVALID_ARG, "grid too large");
  int T[3] = {grid->dim == 2 ? 8 : 4, grid->dim == 2 ? 8 : 4, grid->dim == 2 ? 1 : 4};
  if (tile_host)
    for (int a = 0; a < grid->dim; ++a)
      if (tile_host[a] > 0) T[a] = tile_host[a];
  {
    // bins: whole tiles over the cells, tile-major
    int64_t nk = 1;
    for (int a = 0; a < grid->dim; ++a) {
      if (T[a] > 1024) return fail(ctx, OSMPM_E_INVALID_ARG, "tile too large for LDS");
      nk *= (((int64_t)grid->n_nodes[a] - 2 + T[a] - 1) / T[a]) * T[a];
    }
    if (nk > kMaxItems) return fail(ctx, OSMPM_E_INVALID_ARG, "grid too large for its tiles");
  }
  auto *d = new osmpm_domain();
  d->ctx = ctx;
  d->uid = ctx->next_uid++;
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
  osmpm_status s = OSMPM_OK;
  auto part_alloc = [&](PartPtrs &p) {
    if (!s) s = dalloc(d, &p.x, cap * D);
    if (!s) s = dalloc_bytes(ctx, d->allocs, &p.v, cap * D * d->tb);
    if (!s) s = dalloc_bytes(ctx, d->allocs, &p.B, cap * D * D * d->tb);
    if (!s) s = dalloc_bytes(ctx, d->allocs, &p.F, cap * D * D * d->tb);
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
  if (!s) s = dalloc(d, &d->d_cur, 1);
  if (!s) s = dalloc(d, &d->key, cap);
  if (!s) s = dalloc(d, &d->perm, cap);
  if (!s) s = dalloc(d, &d->lperm, cap);
  if (!s) s = dalloc(d, &d->count, (size_t)d->nk + 1);
  if (!s) s = dalloc(d, &d->cell_start, (size_t)d->nk + 1);
  if (!s) s = dalloc(d, &d->cursor, (size_t)d->nk + 1);
  if (!s) s = dalloc(d, &d->tcount, (size_t)d->tg.ntiles + 1);
  if (!s) s = dalloc(d, &d->tl, (size_t)d->tg.nblocks);
  if (!s) s = dalloc(d, &d->nlist, (size_t)nn);
  if (!s) s = dalloc(d, &d->ncnt, (size_t)blocks_for(nn));
  if (!s) s = dalloc(d, &d->lcnt, 2);
  if (!s) s = dalloc(d, &d->m, nn);
  if (!s) s = dalloc(d, &d->vn, nd);
  if (!s) s = dalloc(d, &d->u, nd);
  if (!s) s = dalloc(d, &d->vbc, nd);
  if (!s) s = dalloc(d, &d->bcg, nd);
  if (!s) s = dalloc(d, &d->gamma, nn);
  if (!s) s = dalloc(d, &d->recv, nn);
  if (!s) s = dalloc(d, &d->flink, (size_t)2 * nn);
  if (!s) s = dalloc(d, &d->fr, nd);
  if (!s) s = dalloc(d, &d->q_all, nn);
  if (!s) s = dalloc(d, &d->q_bnd, nn);
  if (!s) s = dalloc(d, &d->qg, (size_t)nn * kMaxGroups);
  if (!s) s = dalloc(d, &d->gg, nd);
  if (!s) s = dalloc_bytes(ctx, d->allocs, &d->gd, nd * d->tb);
  for (void **v : {&d->cr[0], &d->cr[1], &d->cs[0], &d->cs[1], &d->cw[0], &d->cw[1], &d->cw[2], &d->cu, &d->cp,
                   &d->del})
    if (!s) s = dalloc_bytes(ctx, d->allocs, v, nd * d->tb);
  if (!s) s = dalloc_bytes(ctx, d->allocs, &d->Atil, cap * ns * d->tb);
  if (!s) s = dalloc(d, &d->pnum, nd);
  if (!s) s = dalloc(d, &d->pden, nn);
  if (!s) s = dalloc(d, &d->w0, nd);
  if (!s) s = dalloc(d, &d->w1, nd);
  if (!s) s = dalloc(d, &d->w2, nd);
  if (!s) s = dalloc(d, &d->w3, nd);
  if (!s) s = dalloc(d, &d->mu, 64);
  if (!s) s = dalloc(d, &d->lam, 64);
  if (!s) s = dalloc(d, &d->tau_y, 64);
  if (!s) {
    osmpm_domain *self = d;
    s = group_create(ctx, 1, &self, nullptr, &d->solo);
  }
  if (s) {
    osmpm_domain_destroy(d);
    return s;
  }
  // defined initial contents
  auto zero = [&](void *p, size_t bytes) {
    if (!s && hipMemsetAsync(p, 0, bytes, ctx->stream) != hipSuccess) s = OSMPM_E_DEVICE;
  };
  zero(d->d_cur, sizeof(int));
  zero(d->lcnt, 2 * sizeof(int));
  zero(d->vbc, nd * sizeof(double));
  zero(d->u, nd * sizeof(double));
  zero(d->m, nn * sizeof(double));
  zero(d->vn, nd * sizeof(double));
  zero(d->recv, nn);
  zero(d->gamma, nn);
  zero(d->q_all, nn * sizeof(long long));
  zero(d->q_bnd, nn * sizeof(long long));
  for (double *w : {d->w0, d->w1, d->w2, d->w3}) zero(w, nd * sizeof(double));
  if (!s && hipStreamSynchronize(ctx->stream) != hipSuccess) s = OSMPM_E_DEVICE;
  if (s) {
    osmpm_domain_destroy(d);
    return fail(ctx, s, "device initialisation failed");
  }
  *out = d;
  return OSMPM_OK;
}

void osmpm_domain_destroy(osmpm_domain *dom) {
  if (!dom) return;
  osmpm_ctx *c = dom->ctx;
  if (c) (void)hipStreamSynchronize(c->stream);
  group_free(dom->solo);
  group_free(dom->pair);
  if (c) {
    // groups that hold this domain can no longer run; pair groups of other
    // coarse domains that use it as their fine side are released
    std::vector<osmpm_batch *> gs = c->groups;
    for (osmpm_batch *G : gs)
      for (int s = 0; s < G->sides; ++s)
        for (osmpm_domain *m : G->dom[s])
          if (m == dom) G->dead = true;
  }
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
  d->E_h.resize(n_mat);
  d->nu_h.resize(n_mat);
  for (int i = 0; i < n_mat; ++i) {
    d->E_h[i] = mats[i].E;
    d->nu_h[i] = mats[i].nu;
  }
  return OSMPM_OK;
}

osmpm_status osmpm_domain_set_yield(osmpm_domain *d, int32_t n_mat, const double *tau_y) {
  if (!d || n_mat < 0 || n_mat > 64 || (n_mat > 0 && !tau_y)) return OSMPM_E_INVALID_ARG;
  if (n_mat > 0 && n_mat != d->n_mat)
    return fail(d->ctx, OSMPM_E_INVALID_ARG, "yield table length differs from the material table's");
  std::vector<double> t(64, 0.0);
  bool plastic = false;
  for (int i = 0; i < n_mat; ++i) {
    if (std::isnan(tau_y[i])) return fail(d->ctx, OSMPM_E_INVALID_ARG, "NaN yield stress");
    t[i] = tau_y[i];
    if (tau_y[i] > 0.0 && !std::isinf(tau_y[i])) plastic = true;
  }
  osmpm_ctx *c = d->ctx;
  HIP_TRY(c, hipMemcpyAsync(d->tau_y, t.data(), 64 * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (plastic != d->plastic) {
    d->plastic = plastic;
    d->version += 1;  // the descriptor carries the flag
  }
  return OSMPM_OK;
}

osmpm_status osmpm_domain_set_particles(osmpm_domain *d, int64_t n, const double *x, const double *v, const double *B,
                                        const double *F, const double *mass, const double *vol, const int32_t *mat,
                                        const uint8_t *flags) {
  if (!d || n < 0 || n > d->cap) return OSMPM_E_INVALID_ARG;
  if (n > 0 && (!x || !v || !B || !F || !mass || !vol || !mat || !flags)) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  const int D = d->D;
  PartPtrs &p = d->pb[d->cur];
  d->np = (int)n;
  d->version += 1;
  if (n > 0) {
    const dim3 gb(blocks_for(n * D * D, 2048)), blk(kBlock);
    launch(c, -1, 0, -1, k_aos_to_soa<double>, gb, blk, 0, (int64_t)n, D, x, (double *)p.x, d->cap, 0);
    if (d->precision == OSMPM_MIXED) {
      launch(c, -1, 0, -1, k_aos_to_soa<float>, gb, blk, 0, (int64_t)n, D, v, (float *)p.v, d->cap, 0);
      launch(c, -1, 0, -1, k_aos_to_soa<float>, gb, blk, 0, (int64_t)n, D * D, B, (float *)p.B, d->cap, 0);
      launch(c, -1, 0, -1, k_aos_to_soa<float>, gb, blk, 0, (int64_t)n, D * D, F, (float *)p.F, d->cap, D + 1);
    } else {
      launch(c, -1, 0, -1, k_aos_to_soa<double>, gb, blk, 0, (int64_t)n, D, v, (double *)p.v, d->cap, 0);
      launch(c, -1, 0, -1, k_aos_to_soa<double>, gb, blk, 0, (int64_t)n, D * D, B, (double *)p.B, d->cap, 0);
      launch(c, -1, 0, -1, k_aos_to_soa<double>, gb, blk, 0, (int64_t)n, D * D, F, (double *)p.F, d->cap, D + 1);
    }
    HIP_TRY(c, hipMemcpyAsync(p.mass, mass, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(p.vol, vol, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(p.mat, mat, n * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(p.flags, flags, n * sizeof(uint8_t), hipMemcpyDeviceToDevice, c->stream));
    launch(c, -1, 0, -1, k_iota, dim3(blocks_for(n)), blk, 0, (int)n, p.id);
  }
  d->have_p2g = false;
  return check_launch(c);
}

osmpm_status osmpm_domain_set_selection(osmpm_domain *d, double m_ref, double tau) {
  if (!d || !(m_ref > 0.0) || !(tau >= 0.0)) return OSMPM_E_INVALID_ARG;
  if (d->m_ref != m_ref || d->tau != tau) d->version += 1;
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
  if (std::memcmp(&bc, &d->bc, sizeof(SceneBC)) != 0) d->version += 1;
  d->bc = bc;
  return OSMPM_OK;
}

osmpm_status osmpm_p2g(osmpm_domain *d) {
  if (!d) return OSMPM_E_INVALID_ARG;
  return DISPATCH2(d->D, d->precision, p2g_solo)(d);
}

osmpm_status osmpm_implicit_solve(osmpm_domain *d, double dt, int32_t use_schwarz_bc, const osmpm_solve_opts *o,
                                  osmpm_solve_stats *st) {
  if (!d || !o) return OSMPM_E_INVALID_ARG;
  if (o->max_newton < 0 || o->max_cg < 0 || o->max_ls < 0 || !(o->forcing >= 0.0)) return OSMPM_E_INVALID_ARG;
  if (!(dt > 0.0)) return fail(d->ctx, OSMPM_E_INVALID_ARG, "dt must be positive");
  if (!d->have_p2g) return fail(d->ctx, OSMPM_E_STATE, "solve before p2g");
  return DISPATCH2(d->D, d->precision, solve_solo)(d, dt, use_schwarz_bc, o, st);
}

osmpm_status osmpm_g2p(osmpm_domain *d, double dt) {
  if (!d || !(dt > 0.0)) return OSMPM_E_INVALID_ARG;
  if (!d->have_p2g) return fail(d->ctx, OSMPM_E_STATE, "g2p before p2g");
  if (!d->have_solve) return fail(d->ctx, OSMPM_E_STATE, "g2p before an implicit solve of the last p2g's grid");
  return DISPATCH2(d->D, d->precision, g2p_solo)(d, dt);
}

osmpm_status osmpm_interface_build(osmpm_domain *B, osmpm_domain *S, int32_t *n_amb) {
  if (!pair_ok(B, S)) return OSMPM_E_INVALID_ARG;
  if (!B->have_p2g || !S->have_p2g) return fail(B->ctx, OSMPM_E_STATE, "interface before p2g");
  osmpm_batch *G = nullptr;
  osmpm_status s = pair_group(B, S, &G);
  if (s) return s;
  DISPATCH(B->D, interface_group)(G);
  if ((s = read_status(G))) return s;
  if (n_amb) *n_amb = h_int(G, G->off_amb)[0];
  return OSMPM_OK;
}

osmpm_status osmpm_project_S_to_B(osmpm_domain *S, osmpm_domain *B, double eps_tol, const double *vS, double *out) {
  if (!pair_ok(B, S) || !out || !(eps_tol >= 0.0)) return OSMPM_E_INVALID_ARG;
  osmpm_batch *G = nullptr;
  osmpm_status s = pair_group(B, S, &G);
  if (s) return s;
  DISPATCH(B->D, project_group)(G, eps_tol, vS, -1, out);
  return check_launch(B->ctx);
}

osmpm_status osmpm_interp_B_to_S(osmpm_domain *B, const double *vB, osmpm_domain *S, double *out) {
  if (!pair_ok(B, S) || !out) return OSMPM_E_INVALID_ARG;
  osmpm_batch *G = nullptr;
  osmpm_status s = pair_group(B, S, &G);
  if (s) return s;
  DISPATCH(B->D, interp_group)(G, vB ? -1 : kBufVn, vB, -1, out);
  return check_launch(B->ctx);
}

osmpm_status osmpm_temporal_interp(osmpm_ctx *ctx, int64_t n, int32_t m, int32_t M, const double *vn,
                                   const double *vn1, double *out) {
  if (!ctx || n < 0 || M < 1 || m < 0 || m > M || (n > 0 && (!vn || !vn1 || !out))) return OSMPM_E_INVALID_ARG;
  if (n == 0) return OSMPM_OK;
  launch(ctx, -1, 0, -1, k_temporal_1, dim3(blocks_for(n, 4096)), dim3(kBlock), 0, n, (double)m / (double)M, vn, vn1,
         out);
  return check_launch(ctx);
}

osmpm_status osmpm_set_schwarz_bc(osmpm_domain *d, const double *vbc) {
  if (!d || !vbc) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  HIP_TRY(c, hipMemcpyAsync(d->vbc, vbc, (size_t)d->g.nn * d->D * sizeof(double), hipMemcpyDeviceToDevice,
                            c->stream));
  return OSMPM_OK;
}

static bool schwarz_opts_ok(const osmpm_schwarz_opts *o) {
  return o && o->M >= 1 && o->k_max >= 1 && o->eps_tol >= 0.0 && o->coarse.max_newton >= 0 && o->coarse.max_cg >= 0 &&
         o->coarse.max_ls >= 0 && o->fine.max_newton >= 0 && o->fine.max_cg >= 0 && o->fine.max_ls >= 0 &&
         o->coarse.forcing >= 0.0 && o->fine.forcing >= 0.0;
}

osmpm_status osmpm_schwarz_frame(osmpm_domain *B, osmpm_domain *S, double dT, const osmpm_schwarz_opts *o,
                                 osmpm_schwarz_stats *st) {
  if (!pair_ok(B, S) || !schwarz_opts_ok(o) || !(dT > 0.0)) return OSMPM_E_INVALID_ARG;
  osmpm_batch *G = nullptr;
  osmpm_status s = pair_group(B, S, &G);
  if (s) return s;
  return DISPATCH2(B->D, B->precision, schwarz_group)(G, dT, o, st);
}

osmpm_status osmpm_single_frame(osmpm_domain *d, double dt, const osmpm_solve_opts *o, osmpm_solve_stats *st) {
  if (!d || !o || !(dt > 0.0)) return OSMPM_E_INVALID_ARG;
  if (o->max_newton < 0 || o->max_cg < 0 || o->max_ls < 0 || !(o->forcing >= 0.0)) return OSMPM_E_INVALID_ARG;
  return DISPATCH2(d->D, d->precision, single_group)(d->solo, dt, o, st);
}

osmpm_status osmpm_batch_create(osmpm_ctx *ctx, int32_t n, osmpm_domain *const *coarse, osmpm_domain *const *fine,
                                osmpm_batch **out) {
  if (!ctx || !out || !coarse || n < 1) return OSMPM_E_INVALID_ARG;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!coarse[i]) return OSMPM_E_INVALID_ARG;
    if (fine && !pair_ok(coarse[i], fine[i])) return fail(ctx, OSMPM_E_INVALID_ARG, "mismatched coarse/fine pair");
    for (int j = 0; j < i; ++j)
      if (coarse[j] == coarse[i] || (fine && (fine[j] == fine[i] || fine[j] == coarse[i] || coarse[j] == fine[i])))
        return fail(ctx, OSMPM_E_INVALID_ARG, "a domain appears twice in the batch");
  }
  return group_create(ctx, n, coarse, fine, out);
}

osmpm_status osmpm_batch_schwarz_frame(osmpm_batch *b, double dT, const osmpm_schwarz_opts *o,
                                       osmpm_schwarz_stats *stats) {
  if (!b || b->sides != 2 || !schwarz_opts_ok(o) || !(dT > 0.0)) return OSMPM_E_INVALID_ARG;
  if (b->multi) return fail(b->c, OSMPM_E_INVALID_ARG, "a multi-domain group takes osmpm_multi_schwarz_frame");
  return DISPATCH2(b->D, b->precision, schwarz_group)(b, dT, o, stats);
}

osmpm_status osmpm_multi_create(osmpm_ctx *ctx, osmpm_domain *coarse, int32_t k, osmpm_domain *const *fine,
                                osmpm_batch **out) {
  if (!ctx || !out || !coarse || !fine || k < 1 || k > 1024) return OSMPM_E_INVALID_ARG;
  *out = nullptr;
  for (int i = 0; i < k; ++i) {
    if (!pair_ok(coarse, fine[i])) return fail(ctx, OSMPM_E_INVALID_ARG, "mismatched coarse/fine domain");
    for (int j = 0; j < i; ++j)
      if (fine[j] == fine[i]) return fail(ctx, OSMPM_E_INVALID_ARG, "a fine domain appears twice");
  }
  std::vector<osmpm_domain *> side0((size_t)k, coarse);
  osmpm_status s = group_create(ctx, k, side0.data(), fine, out);
  if (!s) (*out)->multi = true;
  return s;
}

osmpm_status osmpm_multi_schwarz_frame(osmpm_batch *b, double dT, const osmpm_schwarz_opts *o,
                                       osmpm_schwarz_stats *stats) {
  if (!b || b->sides != 2 || !schwarz_opts_ok(o) || !(dT > 0.0)) return OSMPM_E_INVALID_ARG;
  if (!b->multi) return fail(b->c, OSMPM_E_INVALID_ARG, "not a multi-domain group");
  return DISPATCH2(b->D, b->precision, schwarz_multi)(b, dT, o, stats);
}

osmpm_status osmpm_batch_single_frame(osmpm_batch *b, double dt, const osmpm_solve_opts *o,
                                      osmpm_solve_stats *stats) {
  if (!b || b->sides != 1 || !o || !(dt > 0.0)) return OSMPM_E_INVALID_ARG;
  if (o->max_newton < 0 || o->max_cg < 0 || o->max_ls < 0 || !(o->forcing >= 0.0)) return OSMPM_E_INVALID_ARG;
  return DISPATCH2(b->D, b->precision, single_group)(b, dt, o, stats);
}

osmpm_status osmpm_batch_run(osmpm_batch *b, int32_t n_frames, double dT, const osmpm_schwarz_opts *o,
                             int32_t checkpoint_every, const double *bc_host, osmpm_schwarz_stats *stats) {
  if (!b || b->sides != 2 || !schwarz_opts_ok(o) || !(dT > 0.0) || n_frames < 1 || checkpoint_every < 1)
    return OSMPM_E_INVALID_ARG;
  if (b->multi) return fail(b->c, OSMPM_E_INVALID_ARG, "a multi-domain group has no multi-frame run");
  osmpm_status s = group_sync(b);
  if (s) return s;
  return DISPATCH2(b->D, b->precision, batch_run_impl)(b, n_frames, dT, o, checkpoint_every, bc_host, stats);
}

osmpm_status osmpm_batch_backward(osmpm_batch *b, const double *const *xbar_B_host,
                                  const double *const *xbar_S_host, double adj_cg_rtol, int32_t mode, double fp_tol,
                                  int32_t fp_max, double *dL_dE_host) {
  if (!b || b->sides != 2 || !dL_dE_host || !(adj_cg_rtol > 0.0) || (mode != 0 && mode != 1))
    return OSMPM_E_INVALID_ARG;
  if (mode == 1 && (fp_max < 1 || std::isnan(fp_tol))) return OSMPM_E_INVALID_ARG;
  if (!b->run) return fail(b->c, OSMPM_E_STATE, "no osmpm_batch_run to differentiate");
  for (int i = 0; i < b->n; ++i)
    for (int sd = 0; sd < 2; ++sd)
      if (b->dom[sd][i]->plastic) return fail(b->c, OSMPM_E_INVALID_ARG, kNoPlasticAdjoint);
  for (int i = 0; i < b->n; ++i)
    for (int sd = 0; sd < 2; ++sd)
      if (b->dom[sd][i]->n_mat < 1 || (int)b->dom[sd][i]->nu_h.size() != b->dom[sd][i]->n_mat)
        return fail(b->c, OSMPM_E_STATE, "a domain has no material table");
  osmpm_status s = group_sync(b);
  if (s) return s;
  return DISPATCH2(b->D, b->precision, batch_backward_impl)(b, xbar_B_host, xbar_S_host, adj_cg_rtol, mode, fp_tol,
                                                            fp_max, dL_dE_host);
}

void osmpm_batch_destroy(osmpm_batch *b) { group_free(b); }

osmpm_status osmpm_single_frame_adjoint(osmpm_domain *d, double dt, const osmpm_solve_opts *o, double adj_cg_rtol,
                                        const double *xbar, const double *vbar, const double *Bbar,
                                        const double *Fbar, double *oxbar, double *ovbar, double *oBbar,
                                        double *oFbar, double *mubar, double *lambar) {
  if (!d || !o || !(dt > 0.0) || !(adj_cg_rtol > 0.0) || !mubar || !lambar) return OSMPM_E_INVALID_ARG;
  if (o->max_newton < 0 || o->max_cg < 0 || o->max_ls < 0 || !(o->forcing >= 0.0)) return OSMPM_E_INVALID_ARG;
  if (d->np > 0 && (!xbar || !vbar || !Bbar || !Fbar || !oxbar || !ovbar || !oBbar || !oFbar))
    return OSMPM_E_INVALID_ARG;
  if (d->plastic) return fail(d->ctx, OSMPM_E_INVALID_ARG, kNoPlasticAdjoint);
  const double *in[4] = {xbar, vbar, Bbar, Fbar};
  double *out[4] = {oxbar, ovbar, oBbar, oFbar};
  Arena A;
  A.c = d->ctx;
  return DISPATCH2(d->D, d->precision, single_adjoint_impl)(d, dt, o, adj_cg_rtol, in, out, mubar, lambar, A);
}

osmpm_status osmpm_single_frame_adjoint_noalloc(osmpm_domain *d, double dt, const osmpm_solve_opts *o,
                                                double adj_cg_rtol, const double *xbar, const double *vbar,
                                                const double *Bbar, const double *Fbar, double *oxbar,
                                                double *ovbar, double *oBbar, double *oFbar, double *mubar,
                                                double *lambar) {
  if (!d || !o || !(dt > 0.0) || !(adj_cg_rtol > 0.0) || !mubar || !lambar) return OSMPM_E_INVALID_ARG;
  if (o->max_newton < 0 || o->max_cg < 0 || o->max_ls < 0 || !(o->forcing >= 0.0)) return OSMPM_E_INVALID_ARG;
  if (d->np > 0 && (!xbar || !vbar || !Bbar || !Fbar || !oxbar || !ovbar || !oBbar || !oFbar))
    return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  if (d->plastic) return fail(c, OSMPM_E_INVALID_ARG, kNoPlasticAdjoint);
  void *region = fixed_region(c->device);
  if (!region) return fail(c, OSMPM_E_DEVICE, "fixed work region not set up on this device");
  const size_t need = single_adjoint_bytes(d);
  if (need > kFixedRegionBytes)
    return fail(c, OSMPM_E_INVALID_ARG, "single-frame adjoint needs " + std::to_string(need) +
                                            " bytes of work arrays; the fixed region holds " +
                                            std::to_string(kFixedRegionBytes));
  const double *in[4] = {xbar, vbar, Bbar, Fbar};
  double *out[4] = {oxbar, ovbar, oBbar, oFbar};
  Arena A;
  A.c = c;
  A.base = static_cast<char *>(region);
  A.cap = kFixedRegionBytes;
  // graph replay (instantiation allocates) and kernel timing (event
  // creation) are suspended for the call
  const int graphs = c->graphs;
  const bool prof = c->prof;
  c->graphs = 0;
  c->prof = false;
  const osmpm_status s =
      DISPATCH2(d->D, d->precision, single_adjoint_impl)(d, dt, o, adj_cg_rtol, in, out, mubar, lambar, A);
  c->graphs = graphs;
  c->prof = prof;
  return s;
}

static osmpm_status schwarz_adjoint_call(osmpm_domain *B, osmpm_domain *S, double dT, const osmpm_schwarz_opts *o,
                                  int32_t iters, double adj_cg_rtol, int implicit, double fp_tol, int32_t fp_max,
                                  int32_t *fp_used, const double *xbB, const double *vbB, const double *BbB,
                                  const double *FbB, const double *xbS, const double *vbS, const double *BbS,
                                  const double *FbS, double *oxB, double *ovB, double *oBB, double *oFB,
                                  double *oxS, double *ovS, double *oBS, double *oFS, double *mubarB,
                                  double *lambarB, double *mubarS, double *lambarS) {
  if (!pair_ok(B, S) || !schwarz_opts_ok(o) || !(dT > 0.0) || iters < 1 || iters > o->k_max ||
      !(adj_cg_rtol > 0.0) || !mubarB || !lambarB || !mubarS || !lambarS)
    return OSMPM_E_INVALID_ARG;
  if (implicit && (fp_max < 1 || std::isnan(fp_tol))) return OSMPM_E_INVALID_ARG;
  if (B->np > 0 && (!xbB || !vbB || !BbB || !FbB || !oxB || !ovB || !oBB || !oFB)) return OSMPM_E_INVALID_ARG;
  if (S->np > 0 && (!xbS || !vbS || !BbS || !FbS || !oxS || !ovS || !oBS || !oFS)) return OSMPM_E_INVALID_ARG;
  if (B->plastic || S->plastic) return fail(B->ctx, OSMPM_E_INVALID_ARG, kNoPlasticAdjoint);
  osmpm_batch *G = nullptr;
  osmpm_status s = pair_group(B, S, &G);
  if (s) return s;
  const double *inB[4] = {xbB, vbB, BbB, FbB}, *inS[4] = {xbS, vbS, BbS, FbS};
  double *outB[4] = {oxB, ovB, oBB, oFB}, *outS[4] = {oxS, ovS, oBS, oFS};
  std::vector<double> mat(256, 0.0);
  int used = 0;
  s = DISPATCH2(B->D, B->precision, schwarz_adjoint_impl)(G, dT, o, iters, adj_cg_rtol, implicit, fp_tol, fp_max,
                                                          &used, inB, inS, outB, outS, mat.data());
  if (fp_used) *fp_used = used;
  if (s) return s;
  for (int k = 0; k < B->n_mat; ++k) {
    mubarB[k] += mat[k];
    lambarB[k] += mat[64 + k];
  }
  for (int k = 0; k < S->n_mat; ++k) {
    mubarS[k] += mat[128 + k];
    lambarS[k] += mat[192 + k];
  }
  return OSMPM_OK;
}
osmpm_status osmpm_schwarz_frame_adjoint(osmpm_domain *B, osmpm_domain *S, double dT, const osmpm_schwarz_opts *o,
                                         int32_t iters, double adj_cg_rtol, const double *xbB, const double *vbB,
                                         const double *BbB, const double *FbB, const double *xbS,
                                         const double *vbS, const double *BbS, const double *FbS, double *oxB,
                                         double *ovB, double *oBB, double *oFB, double *oxS, double *ovS,
                                         double *oBS, double *oFS, double *mubarB, double *lambarB, double *mubarS,
                                         double *lambarS) {
  return schwarz_adjoint_call(B, S, dT, o, iters, adj_cg_rtol, 0, 0.0, 0, nullptr, xbB, vbB, BbB, FbB, xbS, vbS,
                              BbS, FbS, oxB, ovB, oBB, oFB, oxS, ovS, oBS, oFS, mubarB, lambarB, mubarS, lambarS);
}

osmpm_status osmpm_schwarz_frame_adjoint_implicit(
    osmpm_domain *B, osmpm_domain *S, double dT, const osmpm_schwarz_opts *o, int32_t iters, double adj_cg_rtol,
    double fp_tol, int32_t fp_max, int32_t *fp_used, const double *xbB, const double *vbB, const double *BbB,
    const double *FbB, const double *xbS, const double *vbS, const double *BbS, const double *FbS, double *oxB,
    double *ovB, double *oBB, double *oFB, double *oxS, double *ovS, double *oBS, double *oFS, double *mubarB,
    double *lambarB, double *mubarS, double *lambarS) {
  return schwarz_adjoint_call(B, S, dT, o, iters, adj_cg_rtol, 1, fp_tol, fp_max, fp_used, xbB, vbB, BbB, FbB,
                              xbS, vbS, BbS, FbS, oxB, ovB, oBB, oFB, oxS, ovS, oBS, oFS, mubarB, lambarB, mubarS,
                              lambarS);
}

osmpm_status osmpm_get_particles(osmpm_domain *d, double *x, double *v, double *B, double *F, int32_t *id) {
  if (!d) return OSMPM_E_INVALID_ARG;
  osmpm_ctx *c = d->ctx;
  const int D = d->D;
  const int64_t n = d->np;
  if (n == 0) return OSMPM_OK;
  const PartPtrs &p = d->pb[d->cur];
  const dim3 gb(blocks_for(n * D * D, 2048)), blk(kBlock);
  if (x) launch(c, -1, 0, -1, k_soa_to_aos<double>, gb, blk, 0, n, D, (const double *)p.x, d->cap, x, 0);
  if (d->precision == OSMPM_MIXED) {
    if (v) launch(c, -1, 0, -1, k_soa_to_aos<float>, gb, blk, 0, n, D, (const float *)p.v, d->cap, v, 0);
    if (B) launch(c, -1, 0, -1, k_soa_to_aos<float>, gb, blk, 0, n, D * D, (const float *)p.B, d->cap, B, 0);
    if (F) launch(c, -1, 0, -1, k_soa_to_aos<float>, gb, blk, 0, n, D * D, (const float *)p.F, d->cap, F, D + 1);
  } else {
    if (v) launch(c, -1, 0, -1, k_soa_to_aos<double>, gb, blk, 0, n, D, (const double *)p.v, d->cap, v, 0);
    if (B) launch(c, -1, 0, -1, k_soa_to_aos<double>, gb, blk, 0, n, D * D, (const double *)p.B, d->cap, B, 0);
    if (F) launch(c, -1, 0, -1, k_soa_to_aos<double>, gb, blk, 0, n, D * D, (const double *)p.F, d->cap, F, D + 1);
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
