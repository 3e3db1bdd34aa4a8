// Kernel interface shared by kernels.hip and the host orchestration.
//
// Every kernel runs over a batch of domains in one launch: blockIdx.y is the
// domain's index in the batch and a device array of DomDesc describes each
// domain (grid, tiles, buffers).  Domains of uneven size share a launch;
// blocks beyond a domain's own range exit at once, and a domain whose
// `active` flag is clear (or whose solve phase is finished) skips the launch.
// A single domain is a batch of one.
#pragma once

#include "device.hpp"

namespace osmpm {

// Scalars of one preconditioned CG solve in the single-reduction form (each
// iteration applies the previous direction and forms the next residual, its
// preconditioned image u and the product A u together).  Values written by a
// launch are double-buffered by iteration parity so no workgroup overwrites
// what another workgroup of the same launch still reads.
struct CgState {
  double gam[2];  // (r, u) of earlier iterations, by parity
  double alp[2];  // step lengths of earlier iterations, by parity
  double rr0;     // |r_0|^2
  double alpha_n; // split mode: step length and direction weight of the next launch
  double beta_n;
  double eta;     // relative CG tolerance of this Newton step beyond the fixed one (0: none)
  int red_cnt;    // split mode: workgroups of the current k_cg_reduce that have added their share
  int pad;
  int iter;       // directions applied so far
  int done;       // converged, broke down, hit max_cg, or not solving
  int k_at[2];    // iteration index read by a launch of parity q (written for q ^ 1)
};

// Phases of one domain's implicit solve.  The decision kernels move a domain
// through them on the device; every other solve kernel runs only for domains
// in its phase, so the host can queue a fixed cycle of launches for a whole
// batch and read the states once per cycle.
enum : int {
  kPhaseDone = 0,    // converged, stopped, or not solving
  kPhaseGrad = 1,    // gradient and tangents wanted at the current iterate
  kPhaseCgInit = 2,  // Newton continues: CG to be initialised
  kPhaseCg = 3,      // CG iterating
  kPhaseLs = 4,      // line search on the CG direction
  kPhaseStep = 5,    // step accepted: apply it, then the gradient again
};

// Newton / line-search state of one domain's implicit solve.
struct SolveState {
  double gnorm0, gnorm, gscale, alpha, dE;
  double gref;  // reference norm of the Newton test from a warm-start slot, or -1
  int it;  // Newton iteration index
  int phase;
  int ls_count;
  int converged, ls_failed;
  int newton_iters, cg_iters, ls_halvings;
  int n_active;  // nodes with m > 0 after the last P2G
  int n_tiles_live;  // tiles holding particles after the last binning
  // running totals over the solves of a frame (Newton steps, CG iterations,
  // line-search halvings, unconverged solves, failed line searches), kept
  // on the device when a whole Schwarz iteration replays as one graph
  int tally[5];
};

__host__ __device__ inline bool phase_wants_grad(int ph) { return ph == kPhaseGrad || ph == kPhaseStep; }

// Bit set of up to 1024 domains, passed by value to set batch flags.
struct FlagMask {
  uint64_t w[16];
};

// One particle buffer (component-major [rows][capacity]); v, B, F are in
// the domain's bulk type.  The F rows hold the displacement gradient
// H = F - I, not F: at the small strains of stiff or finely resolved domains
// F sits within 1e-4 of the identity, where a 32-bit F would keep only about
// three digits of the strain, while a 32-bit H keeps its relative accuracy
// at any strain.
struct PartPtrs {
  double *x, *mass, *vol;
  void *v, *B, *F;
  int *mat, *id;
  uint8_t *flags;
};

// A workgroup slot of a tile launch: the live tile it takes and that tile's
// particle range (tile -1: none).
struct alignas(16) TileSlot {
  int tile, p0, p1, pad;
};

struct DomDesc {
  GridDev g;
  TileGeom tg;
  SceneBC bc;
  int np, ndof, nk;
  int64_t cap;
  double scale;     // 2^32 / m_ref
  long long tau_q;  // selection threshold in fixed point
  double Dinv;      // 4 / dx^2
  int *cur;         // index of the current particle buffer (domain-owned)
  int *active;      // takes part in batched launches (batch-owned)
  SolveState *ss;   // solve state (batch-owned)
  PartPtrs pb[2], st;
  int *key, *count, *cell_start, *cursor, *perm, *lperm;
  int *tcount;  // per-tile bin totals, then tile offsets [ntiles + 1]
  // Work lists rebuilt after each binning / P2G: tl[b] = {tile, p0, p1, 0} of
  // the live (particle-holding) tile that workgroup b of a tile launch takes
  // ({-1, 0, 0, 0}: none), [nblocks]; nlist = active nodes (m > 0) in node
  // order, [nn]; ncnt = active nodes per block of 256 nodes; lcnt = {live
  // tiles, active nodes}.
  TileSlot *tl;
  int *nlist, *ncnt, *lcnt;
  const double *mu, *lam;
  double *m, *vn, *u, *vbc, *gg;
  int8_t *bcg;
  uint8_t *gamma, *recv, *fr;
  long long *q_all, *q_bnd, *qg;
  void *gd;                // Jacobi diagonal
  void *cr[2], *cs[2];     // residuals r, products s = A p (by parity)
  void *cw[3];             // products w = A u (three-way rotation)
  void *cu, *cp, *del;     // preconditioned residual u, direction p, Newton step
  void *Atil;              // per-particle folded tangents (packed)
  CgState *cg;
  double *part_a, *part_b;  // per-block partial sums (batch-owned)
  double *part_cg;          // CG partials [parity][(r,u), (Au,u), (r,r)][pstride]
  int pstride;
  double *pnum, *pden, *w0, *w1, *w2, *w3;                // interface work buffers
  // Warm-start slots (one per implicit solve of a Schwarz iteration), each
  // [u: ndof][m: nn][reference norm: 1], warm_stride doubles apart; null
  // when the domain has none.
  double *warm;
  int warm_stride;
  // Fine-fine links of a multi group with overlapping refined regions:
  // [node][2] = {donor fine domain, its node}, or {-1, -1}.
  int *flink;
  // von Mises yield stress per material (elastoplastic extension), and
  // whether any material yields (0: G2P skips the projection)
  const double *tau_y;
  int plastic;
};

// Blocks a grid-stride node kernel uses for a domain (also the number of
// partial sums it writes).
__host__ __device__ inline int node_blocks(int ndof) {
  int b = (ndof + kBlock - 1) / kBlock;
  return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

template <typename T>
__global__ void k_fill(int64_t n, T v, T *a);
template <typename T>
__global__ void k_aos_to_soa(int64_t n, int c, const double *src, T *dst, int64_t cap, int eye);
template <typename T>
__global__ void k_soa_to_aos(int64_t n, int c, const T *src, int64_t cap, double *dst, int eye);
__global__ void k_iota(int n, int *a);
__global__ void k_set_flags(int *flags, int n, FlagMask m);
__global__ void k_temporal_1(int64_t n, double am, const double *vn, const double *vn1, double *out);

// binning
template <int D>
__global__ void k_keys(const DomDesc *dd, int *err);
__global__ void k_tile_sum(const DomDesc *dd);
__global__ void k_tile_scan(const DomDesc *dd);
__global__ void k_cell_scan(const DomDesc *dd);
__global__ void k_scatter(const DomDesc *dd);
__global__ void k_cellsort(const DomDesc *dd);
__global__ void k_slot_layout(const DomDesc *dd);
__global__ void k_flip(const DomDesc *dd, int ndom);
template <int D, typename TB>
__global__ void k_copy_state(const DomDesc *dd, int to_store);
__global__ void k_zero_grid(const DomDesc *dd, int want_q);

// transfers
template <int D, typename TB, bool kQ>
__global__ void k_p2g(const DomDesc *dd, int *err);
template <int D>
__global__ void k_p2g_final(const DomDesc *dd);
template <int D, typename TB>
__global__ void k_g2p(const DomDesc *dd, double dt, int *err);
template <int D, typename TB>
__global__ void k_plastic_return(const DomDesc *dd);

// implicit solve
template <int D, typename TB>
__global__ void k_bc_init(const DomDesc *dd, double dt, int use_schwarz, int vbc_buf, int warm_slot);
__global__ void k_solve_begin(const DomDesc *dd, double dt, int warm_slot);
__global__ void k_warm_keep(const DomDesc *dd, int slot, int first);
__global__ void k_solve_tally(const DomDesc *dd, int reset);
template <int D, typename TB>
__global__ void k_grad_hess(const DomDesc *dd, int project, int *err);
template <int D, typename TB>
__global__ void k_grad_node(const DomDesc *dd, double dt, double gx, double gy, double gz);
template <int D, typename TB>
__global__ void k_cg_init(const DomDesc *dd, int check, double rtol, double atol, int max_newton, double forcing);
template <int D, typename TB>
__global__ void k_cg_iter(const DomDesc *dd, int q, double dt, double rtol, int max_cg, int split);
__global__ void k_tile_list(const DomDesc *dd);
__global__ void k_node_count(const DomDesc *dd);
// Node blocks (of kBlock nodes) up to which k_node_list forms each block's
// offset from the per-block counts itself; larger grids scan the counts
// first with k_node_scan.
constexpr int kNodeListDirect = 1024;
__global__ void k_node_scan(const DomDesc *dd);
__global__ void k_node_list(const DomDesc *dd);
// Workgroups of a CG launch that do work: one per live-tile slot (whole
// bands of 8) and enough for the active DOFs, at least one, at most the
// domain's tile blocks.  The lists do not change during a solve, so every
// launch of it (and the split-mode reduction) derives the same count; the
// host sizes large launches with the same formula.
__host__ __device__ inline int cg_work_blocks(int live_tiles, int active_dofs, int nblocks) {
  int nw = ((live_tiles + 7) >> 3) * 8;
  const int nown = (active_dofs + kBlock - 1) / kBlock;
  nw = nw > nown ? nw : nown;
  nw = nw > 1 ? nw : 1;
  return nw < nblocks ? nw : nblocks;
}

// Workgroups per domain of k_cg_reduce for launches of up to `tile_blocks`
// workgroups (one up to 8192, at most 256).
inline int cg_reduce_blocks(int tile_blocks) {
  const int r = tile_blocks / 4096;
  return r < 1 ? 1 : (r > 256 ? 256 : r);
}
__global__ void k_cg_reduce(const DomDesc *dd, int q, double rtol, int max_cg);
template <int D, typename TB>
__global__ void k_delta_energy(const DomDesc *dd, double dt, double gx, double gy, double gz);
__global__ void k_ls_check(const DomDesc *dd, int max_ls);

// interface
template <int D>
__global__ void k_qbnd(const DomDesc *dd);
__global__ void k_gamma(const DomDesc *dd);
__global__ void k_count_recv(const DomDesc *dd, int *out);
template <int D>
__global__ void k_arbitrate(const DomDesc *ddB, const DomDesc *ddS, int *n_amb);
__global__ void k_zero_proj(const DomDesc *ddB);
template <int D>
__global__ void k_project_scatter(const DomDesc *ddS, const DomDesc *ddB, const double *vS_ext, int *err);
template <int D>
__global__ void k_project_final(const DomDesc *ddB, double eps_tol, int which, double *out_ext);
template <int D>
__global__ void k_interp(const DomDesc *ddB, const DomDesc *ddS, int src, const double *vB_ext, int dst,
                         double *out_ext, int *err);
template <int D>
__global__ void k_temporal(const DomDesc *dd, double am, int a_buf, int b_buf);
template <int D>
__global__ void k_vel_from_u(const DomDesc *dd, double dt);
template <int D>
__global__ void k_fine_arbitrate(const DomDesc *dd, int n, int *n_amb);
template <int D>
__global__ void k_fine_links(const DomDesc *dd, int n);
template <int D>
__global__ void k_fine_link_apply(const DomDesc *dd, int slot, double dt, int dst_buf);
template <int D>
__global__ void k_resid(const DomDesc *dd, int a_buf, int b_buf);
template <int D>
__global__ void k_copy_vbc(const DomDesc *dd, int src);
__global__ void k_resid_final(const DomDesc *dd, double *out);

// reverse mode (adjoint.hip)
template <int D, typename TB>
__global__ void k_adj_p2g(GridDev g, int np, int64_t cap, const double *x, const TB *v, const TB *B,
                          const double *mass, const int *id, const double *m, const double *vn, const double *mbar,
                          const double *vnbar, double *ax, double *av, double *aB);
template <int D, typename TB>
__global__ void k_adj_g2p(GridDev g, int np, int64_t cap, const double *x, const TB *F, const int *id,
                          const double *m, const double *u, double dt, const double *ix, const double *iv,
                          const double *iB, const double *iF, double *ubar, double *ox, double *oF);
__global__ void k_adj_set_rhs(const DomDesc *dd, const double *ubar);
template <int D, typename TB>
__global__ void k_adj_hvp(const DomDesc *dd, const TB *lam, double *y);
template <int D, typename TB>
__global__ void k_adj_solve_nodes(const DomDesc *dd, double dt, double gx, double gy, double gz, const double *ubar,
                                  const double *hl, int use_schwarz, double *mbar, double *vnbar, double *vbcbar);
template <int D, typename TB>
__global__ void k_adj_solve_particles(const DomDesc *dd, double *ax, double *aF, int np_adj, double *mubar,
                                      double *lambar);
template <int D>
__global__ void k_adj_project(GridDev gB, GridDev gS, const double *mS, const double *vnS, const uint8_t *recvB,
                              const double *num, const double *den, double eps_tol, const double *pbar,
                              double *mbarS, double *vnbarS);
template <int D>
__global__ void k_adj_interp(GridDev gB, GridDev gS, const double *mB, const uint8_t *recvS, const double *ibar,
                             double *vBbar);
__global__ void k_adj_temporal(int64_t n, double am, const double *vbcbar, double *a, double *b);
__global__ void k_axpy_d(int64_t n, double a, const double *x, double *y);
__global__ void k_sumsq_d(int64_t n, const double *x, double *out);
template <int D>
__global__ void k_adj_vel(int nn, const double *m, const double *vbar, double dT, double *ubar);

// Work buffer selector of the interface kernels.
__device__ inline double *wbuf(const DomDesc &D, int k) {
  switch (k) {
    case 0: return D.w0;
    case 1: return D.w1;
    case 2: return D.w2;
    case 3: return D.w3;
    case 4: return D.vn;
    default: return D.vbc;
  }
}

}  // namespace osmpm
