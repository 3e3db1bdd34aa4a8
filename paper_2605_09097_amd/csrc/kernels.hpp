// Kernel declarations shared by kernels.hip and the host orchestration.
#pragma once

#include "device.hpp"

namespace osmpm {

// Scalars of one CG solve, kept on the device between the two kernels of an
// iteration.  rz is double-buffered by iteration parity so a kernel never
// overwrites the value other workgroups of the same launch still read.
struct CgState {
  double rz[2];
  double rr0;
  double pad;
  int iter;   // completed updates
  int done;   // converged, broke down or hit max_cg
  int knext;  // index of the next iteration (written by the update kernel)
  int kcur;   // index of the running iteration (written by the product kernel)
};

template <typename T>
__global__ void k_fill(int64_t n, T v, T *a);
__global__ void k_fill_i64(int64_t n, long long *a);
__global__ void k_fill_i32(int64_t n, int v, int *a);
__global__ void k_fill_u8(int64_t n, uint8_t *a);
template <typename T>
__global__ void k_aos_to_soa(int64_t n, int c, const double *src, T *dst, int64_t cap);
template <typename T>
__global__ void k_soa_to_aos(int64_t n, int c, const T *src, int64_t cap, double *dst);
__global__ void k_iota(int n, int *a);

template <int D>
__global__ void k_keys(int n, const double *x, int64_t cap, GridDev g, TileGeom tg, int *key, int *count, int *err);
__global__ void k_scan(int nk, const int *count, int *cell_start, int *cursor);
__global__ void k_scatter(int n, const int *key, int *cursor, int *perm);
__global__ void k_cellsort(int nk, const int *cell_start, int *perm);
template <typename T>
__global__ void k_gather(int n, int rows, const int *perm, const T *src, T *dst, int64_t cap);

template <int D, typename TB>
__global__ void k_p2g(TileGeom tg, GridDev g, const int *cell_start, const double *x, const TB *v, const TB *B,
                      const double *mass, const uint8_t *flags, int64_t cap, int n_groups, double scale, double Dinv,
                      int want_q, double *gm, double *gmv, long long *q_all, long long *qg, int *err);
template <int D>
__global__ void k_p2g_final(GridDev g, const double *gm, double *gv, const long long *qg, SceneBC bc,
                            long long tau_q, int8_t *bcg);
template <int D, typename TB>
__global__ void k_g2p(int n, GridDev g, const double *gm, const double *u, double dt, double *x, TB *v, TB *B, TB *F,
                      int64_t cap, int *err);

template <int D>
__global__ void k_bc_init(GridDev g, const double *gm, const double *gv, const int8_t *bcg, const uint8_t *recv,
                          const double *vbc, int use_schwarz, SceneBC bc, double dt, uint8_t *fr, double *u,
                          double *part_m);
template <int D, typename TB>
__global__ void k_grad_hess(TileGeom tg, GridDev g, const int *cell_start, const double *x, const TB *F,
                            const double *vol, const int *mat, const double *mu_t, const double *lam_t, int64_t cap,
                            const double *u, int want_hess, int project, double *gg, TB *gdiag, TB *Atil, int *err);
template <int D, typename TB>
__global__ void k_grad_node(GridDev g, const double *gm, const double *gv, const double *u, const uint8_t *fr,
                            double dt, double gx, double gy, double gz, double *gg, TB *gdiag, int want_hess,
                            double *part);
template <int D, typename TB>
__global__ void k_cg_init(int ndof, const double *gg, const TB *gdiag, const uint8_t *fr, TB *r, TB *z, TB *p0,
                          TB *p1, TB *del, TB *Hp, double *part_rz, double *part_rr, CgState *S);
template <int D, typename TB>
__global__ void k_cg_hvp(TileGeom tg, GridDev g, const int *cell_start, const double *x, const TB *Atil, int64_t cap,
                         const double *gm, double dt, int ndof, const TB *z, TB *pA, TB *pB, TB *Hp,
                         const double *part_rz, const double *part_rr, int n_part, double rtol, int max_cg,
                         double *part_q, CgState *S);
template <int D, typename TB>
__global__ void k_cg_update(int ndof, const double *gm, double dt, const uint8_t *fr, const TB *gdiag, const TB *pA,
                            const TB *pB, TB *Hp, TB *r, TB *z, TB *del, const double *part_q, int n_q,
                            double *part_rz, double *part_rr, CgState *S);
template <int D, typename TB>
__global__ void k_delta_energy_p(int np, GridDev g, const double *x, const TB *F, const double *vol, const int *mat,
                                 const double *mu_t, const double *lam_t, int64_t cap, const double *u, const TB *del,
                                 double alpha, double *part);
template <int D, typename TB>
__global__ void k_delta_energy_n(GridDev g, const double *gm, const double *gv, const double *u, const TB *del,
                                 double dt, double alpha, double gx, double gy, double gz, double *part);
template <typename TB>
__global__ void k_axpy(int n, double alpha, const TB *xv, double *y);

template <int D>
__global__ void k_qbnd(int np, GridDev g, const double *x, const double *mass, const uint8_t *flags, int64_t cap,
                       double scale, long long *q_bnd);
__global__ void k_gamma(int nn, const long long *q_bnd, const double *gm, long long tau_q, uint8_t *gamma,
                        uint8_t *recv);
template <int D>
__global__ void k_arbitrate(GridDev gB, GridDev gS, const uint8_t *gammaB, const uint8_t *gammaS,
                            const long long *qB, const long long *qS, uint8_t *recvB, uint8_t *recvS, int *n_amb);
template <int D>
__global__ void k_project_scatter(GridDev gS, GridDev gB, const double *mS, const double *vS, double *num,
                                  double *den, int *err);
template <int D>
__global__ void k_project_final(int nn, const uint8_t *recv, const double *num, const double *den, double eps_tol,
                                double *out);
template <int D>
__global__ void k_interp(GridDev gB, GridDev gS, const double *mB, const double *vB, const uint8_t *recvS,
                         double *out, int *err);
__global__ void k_temporal(int64_t n, double am, const double *vn, const double *vn1, double *out);
template <int D>
__global__ void k_vel_from_u(int nn, const double *gm, const double *u, double dt, double *v);
template <int D>
__global__ void k_resid(int nn, const uint8_t *recv, const double *a, const double *b, double *part);

}  // namespace osmpm
