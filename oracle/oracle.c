/*
 * OS-MPM FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded double-precision implementation of the
 * overlapping-Schwarz material point method (arXiv 2605.09097): APIC
 * particle-to-grid transfer, the backward-Euler incremental potential
 * minimised by Newton's method with Jacobi-preconditioned CG and a halving
 * line search, APIC grid-to-particle transfer with the deformation-gradient
 * update and advection, boundary-grid selection, overlap arbitration, the
 * mass-weighted projection, the coarse-to-fine interpolation, the temporal
 * interpolation and the multiplicative Schwarz frame.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library and must never be used as a fallback for it.
 *
 * Every function names the section / equation of the paper it follows.
 * Readings of passages the paper leaves open are stated where they are used
 * and listed together in the design notes of the repository.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no OpenMP, no intrinsics).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG 1
#define OR_E_NOMEM 2
#define OR_E_OUT_OF_GRID 4
#define OR_E_INVERTED 5
#define OR_E_NOT_CONVERGED 6

#define BC_FIX 0
#define BC_TRANSLATE 1
#define BC_ROTATE 2

/* ------------------------------------------------------------------ */
/* Data                                                                */
/* ------------------------------------------------------------------ */

/* One subdomain: its structured grid (an integer lattice of pitch h0),
 * its particles and its grid state.  All arrays are owned by the caller.
 * Particle arrays are row-major per particle: x[p*d+a], F[p*d*d+a*d+b]. */
typedef struct {
  int dim;
  int n[3];               /* nodes per axis (n[2] == 1 in 2D) */
  double h0;              /* lattice pitch */
  long long origin_q[3];  /* grid origin in lattice units */
  long long dx_q;         /* grid spacing in lattice units */

  int np;
  double *x, *v, *B, *F;  /* particle state, updated in place */
  double *mass, *vol;     /* m_p and V_p^0 */
  int *mat;               /* material index */
  unsigned char *flags;   /* bit0: Schwarz boundary particle; bit 1+g: scene group g */

  int n_mat;
  double *mu, *lam;       /* Lame parameters per material */

  int n_groups;
  int *bc_kind;           /* BC_FIX / BC_TRANSLATE / BC_ROTATE */
  int *bc_mask;           /* component mask */
  double *bc_param;       /* [n_groups][8] */

  double m_ref;           /* unit of the fixed-point node masses: m_ref / 2^32 */
  double tau;             /* selection threshold (a mass) */

  /* grid state, caller-allocated */
  double *m;              /* [nn]     lumped node mass */
  double *vn;             /* [nn][d]  node velocity from P2G */
  double *u;              /* [nn][d]  displacement unknown x_hat - x */
  signed char *bcg;       /* [nn][d]  scene-BC group constraining the DOF, or -1 */
  long long *q_all;       /* [nn]     fixed-point node mass, all particles */
  long long *q_bnd;       /* [nn]     fixed-point node mass, boundary particles */
  unsigned char *gamma;   /* [nn]     boundary grid set */
  unsigned char *recv;    /* [nn]     receiver set after arbitration */
  double *vbc;            /* [nn][d]  Schwarz Dirichlet velocity on receivers */
  int use_schwarz_bc;
  double *tau_y;          /* [n_mat] von Mises yield stress, or NULL: every material elastic
                           * (an entry <= 0 or infinite: that material elastic) */
} or_domain;

typedef struct {
  double newton_rtol, newton_atol, cg_rtol;
  int max_newton, max_cg, max_ls;
  int project_psd;        /* 1: per-particle PSD projection of dP/dF */
  double gravity[3];
} or_solve_opts;

typedef struct {
  int newton_iters, cg_iters, ls_halvings, converged, ls_failed;
  double gnorm0, gnorm, energy;
} or_solve_stats;

typedef struct {
  int M, k_max;
  double eps_conv, eps_tol;
  or_solve_opts coarse, fine;
  int force_iters;        /* > 0: run exactly this many Schwarz iterations */
  int warm_start;         /* 1: Schwarz iterations after the first start each solve from the last one's */
} or_schwarz_opts;

typedef struct {
  int iters, converged;
  double r_B, r_S;
  int n_recv_B, n_recv_S, n_amb;
  int newton_B, newton_S, cg_B, cg_S, ls_B, ls_S;
  int unconv_B, unconv_S, lsfail_B, lsfail_S; /* inner solves unconverged / with a failed line search */
} or_schwarz_stats;

/* ------------------------------------------------------------------ */
/* Grid and quadratic B-spline weights                                 */
/* ------------------------------------------------------------------ */

static int nnodes(const or_domain *D) { return D->n[0] * D->n[1] * D->n[2]; }
static double grid_dx(const or_domain *D) { return (double)D->dx_q * D->h0; }
static int node_flat(const or_domain *D, const int *i) {
  return i[0] + D->n[0] * (i[1] + D->n[1] * i[2]);
}
static void node_index(const or_domain *D, int flat, int *i) {
  i[0] = flat % D->n[0];
  i[1] = (flat / D->n[0]) % D->n[1];
  i[2] = flat / (D->n[0] * D->n[1]);
}
/* Node position x_i = (origin_q + i * dx_q) * h0 on the integer lattice. */
static void node_pos(const or_domain *D, const int *i, double *x) {
  for (int a = 0; a < D->dim; ++a)
    x[a] = (double)(D->origin_q[a] + (long long)i[a] * D->dx_q) * D->h0;
}

/* Quadratic B-spline support of a point (the nodal shape functions N_i of
 * the structured grid, Sec. 2.2.2).  The paper does not state the order; the
 * quadratic B-spline with a 3^d stencil is used.  base = floor(xi - 1/2),
 * f = xi - base in [1/2, 3/2). */
typedef struct {
  int base[3];
  double f[3];
  double w[3][3], dw[3][3];
} stencil;

static int stencil_at(const or_domain *D, const double *xp, stencil *s) {
  const double dx = grid_dx(D);
  const double inv_dx = 1.0 / dx;
  for (int a = 0; a < 3; ++a) {
    s->base[a] = 0;
    s->f[a] = 0.0;
    for (int k = 0; k < 3; ++k) {
      s->w[a][k] = 0.0;
      s->dw[a][k] = 0.0;
    }
  }
  for (int a = 0; a < D->dim; ++a) {
    const double o = (double)D->origin_q[a] * D->h0;
    const double xi = (xp[a] - o) * inv_dx;
    const double bf = floor(xi - 0.5);
    if (!(bf >= 0.0 && bf <= (double)(D->n[a] - 3))) return OR_E_OUT_OF_GRID;
    const double f = xi - bf;
    const double t0 = 1.5 - f, t1 = f - 1.0, t2 = f - 0.5;
    s->base[a] = (int)bf;
    s->f[a] = f;
    s->w[a][0] = 0.5 * (t0 * t0);
    s->w[a][1] = 0.75 - t1 * t1;
    s->w[a][2] = 0.5 * (t2 * t2);
    s->dw[a][0] = -t0 * inv_dx;
    s->dw[a][1] = -2.0 * t1 * inv_dx;
    s->dw[a][2] = t2 * inv_dx;
  }
  return OR_OK;
}

static int stencil_size(const or_domain *D) { return D->dim == 3 ? 27 : 9; }

/* Stencil node number s (x fastest): its flat node index, N_ip, grad N_ip and
 * x_i - x_p.  N = w_x*w_y (2D), (w_x*w_y)*w_z (3D). */
static void stencil_node(const or_domain *D, const stencil *st, int s, int *flat, double *N,
                         double *gN, double *dxv) {
  int k[3] = {s % 3, (s / 3) % 3, s / 9};
  int idx[3] = {0, 0, 0};
  const double dx = grid_dx(D);
  for (int a = 0; a < D->dim; ++a) {
    idx[a] = st->base[a] + k[a];
    dxv[a] = ((double)k[a] - st->f[a]) * dx;
  }
  *flat = node_flat(D, idx);
  const double wx = st->w[0][k[0]], wy = st->w[1][k[1]];
  const double dwx = st->dw[0][k[0]], dwy = st->dw[1][k[1]];
  if (D->dim == 2) {
    *N = wx * wy;
    gN[0] = dwx * wy;
    gN[1] = wx * dwy;
  } else {
    const double wz = st->w[2][k[2]], dwz = st->dw[2][k[2]];
    *N = (wx * wy) * wz;
    gN[0] = (dwx * wy) * wz;
    gN[1] = (wx * dwy) * wz;
    gN[2] = (wx * wy) * dwz;
  }
}

/* Exported for the B-spline identity pins. */
int or_weights(const or_domain *D, const double *xp, int *flat, double *N, double *gN) {
  stencil st;
  int rc = stencil_at(D, xp, &st);
  if (rc) return rc;
  double dxv[3];
  for (int s = 0; s < stencil_size(D); ++s)
    stencil_node(D, &st, s, &flat[s], &N[s], &gN[3 * s], dxv);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Binning: stable counting sort of particles by the cell of their     */
/* base node, in tile-major key order.                                  */
/* ------------------------------------------------------------------ */

/* Number of keys for a tile shape: base positions per axis are n-2, padded to
 * whole tiles; key = tile_flat * tile_volume + local_flat (x fastest). */
long long or_num_keys(const or_domain *D, const int *tile) {
  long long nk = 1;
  for (int a = 0; a < D->dim; ++a) {
    long long nb = D->n[a] - 2;
    long long nt = (nb + tile[a] - 1) / tile[a];
    nk *= nt * tile[a];
  }
  return nk;
}

static long long bin_key(const or_domain *D, const int *tile, const int *base) {
  long long ntile[3] = {1, 1, 1}, T[3] = {1, 1, 1}, t[3] = {0, 0, 0}, l[3] = {0, 0, 0};
  for (int a = 0; a < D->dim; ++a) {
    T[a] = tile[a];
    ntile[a] = (D->n[a] - 2 + tile[a] - 1) / tile[a];
    t[a] = base[a] / tile[a];
    l[a] = base[a] % tile[a];
  }
  long long tf = t[0] + ntile[0] * (t[1] + ntile[1] * t[2]);
  long long lf = l[0] + T[0] * (l[1] + T[1] * l[2]);
  return tf * (T[0] * T[1] * T[2]) + lf;
}

/* perm[i] = original index of the i-th particle in sorted order (stable);
 * cell_start has num_keys + 1 entries. */
int or_sort(const or_domain *D, const int *tile, int *perm, int *cell_start) {
  const long long nk = or_num_keys(D, tile);
  long long *key = (long long *)malloc(sizeof(long long) * (size_t)(D->np > 0 ? D->np : 1));
  int *next = (int *)malloc(sizeof(int) * (size_t)(nk + 1));
  if (!key || !next) {
    free(key);
    free(next);
    return OR_E_NOMEM;
  }
  for (long long k = 0; k <= nk; ++k) cell_start[k] = 0;
  for (int p = 0; p < D->np; ++p) {
    stencil st;
    if (stencil_at(D, &D->x[p * D->dim], &st)) {
      free(key);
      free(next);
      return OR_E_OUT_OF_GRID;
    }
    key[p] = bin_key(D, tile, st.base);
    cell_start[key[p] + 1] += 1;
  }
  for (long long k = 0; k < nk; ++k) cell_start[k + 1] += cell_start[k];
  for (long long k = 0; k <= nk; ++k) next[k] = cell_start[k];
  for (int p = 0; p < D->np; ++p) perm[next[key[p]]++] = p;
  free(key);
  free(next);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* APIC particle-to-grid (Eq. p2g_transfer, Sec. 2.2.4; Eq. p2g_substep) */
/* ------------------------------------------------------------------ */

static double fixed_scale(const or_domain *D) { return 4294967296.0 / D->m_ref; }

/* Fixed-point node mass contribution: rint(N_ip * (m_p * 2^32 / m_ref)).  Node
 * selection sums these as integers so the selected sets do not depend on the
 * order of summation (reading of the "small mass threshold" of Sec. 3.2.1). */
static long long fixed_mass(double N, double mq) { return llrint(N * mq); }

/* m_i = sum m_p N_ip; (mv)_i = sum m_p N_ip (v_p + B_p D_p^-1 (x_i - x_p)) with
 * the quadratic-B-spline inertia tensor D_p = (dx^2/4) I (APIC); v_i = (mv)_i/m_i
 * on nodes with m_i > 0 (the active set).  Also builds the fixed-point node
 * mass of all particles (arbitration, Eq. overlap_donor) and selects the
 * scene-BC nodes of each particle group. */
int or_p2g(or_domain *D) {
  const int d = D->dim, nn = nnodes(D), ss = stencil_size(D);
  const double dx = grid_dx(D), inv_dx = 1.0 / dx;
  const double Dinv = 4.0 * inv_dx * inv_dx;
  const double scale = fixed_scale(D);
  const long long tau_q = llrint(D->tau * scale);
  long long *qg = NULL;
  if (D->n_groups > 0) {
    qg = (long long *)calloc((size_t)D->n_groups * (size_t)nn, sizeof(long long));
    if (!qg) return OR_E_NOMEM;
  }
  for (int i = 0; i < nn; ++i) {
    D->m[i] = 0.0;
    D->q_all[i] = 0;
    for (int a = 0; a < d; ++a) {
      D->vn[i * d + a] = 0.0;
      D->bcg[i * d + a] = -1;
    }
  }
  for (int p = 0; p < D->np; ++p) {
    stencil st;
    if (stencil_at(D, &D->x[p * d], &st)) {
      free(qg);
      return OR_E_OUT_OF_GRID;
    }
    const double mp = D->mass[p];
    const double mq = mp * scale;
    const double *vp = &D->v[p * d];
    const double *Bp = &D->B[p * d * d];
    for (int s = 0; s < ss; ++s) {
      int i;
      double N, gN[3], dxv[3];
      stencil_node(D, &st, s, &i, &N, gN, dxv);
      const double mN = mp * N;
      D->m[i] += mN;
      for (int a = 0; a < d; ++a) {
        double aff = 0.0;
        for (int b = 0; b < d; ++b) aff += Bp[a * d + b] * dxv[b];
        D->vn[i * d + a] += mN * (vp[a] + Dinv * aff);
      }
      const long long q = fixed_mass(N, mq);
      D->q_all[i] += q;
      for (int g = 0; g < D->n_groups; ++g)
        if (D->flags[p] & (2u << g)) qg[(size_t)g * nn + i] += q;
    }
  }
  for (int i = 0; i < nn; ++i) {
    if (D->m[i] > 0.0)
      for (int a = 0; a < d; ++a) D->vn[i * d + a] /= D->m[i];
    for (int a = 0; a < d; ++a) {
      for (int g = 0; g < D->n_groups; ++g) {
        if ((D->bc_mask[g] >> a) & 1) {
          if (qg[(size_t)g * nn + i] > tau_q && D->m[i] > 0.0) {
            D->bcg[i * d + a] = (signed char)g;
            break;
          }
        }
      }
    }
  }
  free(qg);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Compressible Neo-Hookean energy (Sec. 4: "Neo-Hookean"; the paper    */
/* gives no formula).  Psi = mu/2 (|F|^2 - d) - mu ln J + lam/2 (ln J)^2, */
/* which in 2D is the plane-strain energy of diag(F, 1) (Sec. 4.3).      */
/* ------------------------------------------------------------------ */

static double det_d(const double *F, int d) {
  if (d == 2) return F[0] * F[3] - F[1] * F[2];
  return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
         F[2] * (F[3] * F[7] - F[4] * F[6]);
}

/* Cofactor matrix: cof(F)_ij = dJ/dF_ij. */
static void cofactor(const double *F, int d, double *C) {
  if (d == 2) {
    C[0] = F[3];
    C[1] = -F[2];
    C[2] = -F[1];
    C[3] = F[0];
    return;
  }
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

/* Psi(F); +inf when J <= 0. */
static double nh_psi(const double *F, int d, double mu, double lam) {
  const double J = det_d(F, d);
  if (!(J > 0.0)) return INFINITY;
  const double lnJ = log(J);
  double tr = 0.0;
  for (int k = 0; k < d * d; ++k) tr += F[k] * F[k];
  return 0.5 * mu * (tr - (double)d) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
}

/* First Piola stress P = mu (F - F^-T) + lam ln J F^-T and its derivative
 * A[(ab),(ce)] = dP_ab/dF_ce
 *   = mu d_ac d_be + (mu - lam ln J) Finv_ea Finv_bc + lam Finv_ba Finv_ec. */
static int nh_stress(const double *F, int d, double mu, double lam, double *P, double *A) {
  const double J = det_d(F, d);
  if (!(J > 0.0)) return OR_E_INVERTED;
  const double lnJ = log(J);
  double C[9], Finv[9];
  cofactor(F, d, C);
  /* F^-1 = cof(F)^T / J */
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) Finv[a * d + b] = C[b * d + a] / J;
  if (P)
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        const double FinvT = Finv[b * d + a];
        P[a * d + b] = mu * (F[a * d + b] - FinvT) + lam * lnJ * FinvT;
      }
  if (A) {
    const int n = d * d;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b)
        for (int c = 0; c < d; ++c)
          for (int e = 0; e < d; ++e) {
            double v = 0.0;
            if (a == c && b == e) v += mu;
            v += (mu - lam * lnJ) * Finv[e * d + a] * Finv[b * d + c];
            v += lam * Finv[b * d + a] * Finv[e * d + c];
            A[(a * d + b) * n + (c * d + e)] = v;
          }
  }
  return OR_OK;
}

/* Projection of a symmetric n x n matrix onto the PSD cone: cyclic Jacobi
 * eigendecomposition (Golub & Van Loan, Sec. 8.5), negative eigenvalues set
 * to zero.  A matrix whose eigenvalues are all >= 0 is returned unchanged.
 * The paper does not discuss definiteness of the tangent K (Sec. 2.2.5);
 * projected Newton is the reading used here. */
static void psd_project(double *A, int n) {
  double W[81], V[81];
  memcpy(W, A, sizeof(double) * (size_t)(n * n));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  double diag2 = 0.0;
  for (int i = 0; i < n; ++i) diag2 += W[i * n + i] * W[i * n + i];
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += W[p * n + q] * W[p * n + q];
    if (off <= 1e-32 * diag2 || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = W[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (W[q * n + q] - W[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0);
        const double s = t * c;
        /* W <- W J, V <- V J (columns p, q) */
        for (int k = 0; k < n; ++k) {
          const double wkp = W[k * n + p], wkq = W[k * n + q];
          W[k * n + p] = c * wkp - s * wkq;
          W[k * n + q] = s * wkp + c * wkq;
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
        /* W <- J^T W (rows p, q) */
        for (int k = 0; k < n; ++k) {
          const double wpk = W[p * n + k], wqk = W[q * n + k];
          W[p * n + k] = c * wpk - s * wqk;
          W[q * n + k] = s * wpk + c * wqk;
        }
      }
  }
  int neg = 0;
  for (int i = 0; i < n; ++i)
    if (W[i * n + i] < 0.0) neg = 1;
  if (!neg) return;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) {
        const double lk = W[k * n + k] > 0.0 ? W[k * n + k] : 0.0;
        v += V[i * n + k] * lk * V[j * n + k];
      }
      A[i * n + j] = v;
    }
}

/* Exported for the constitutive pins. */
int or_nh_eval(int d, const double *F, double mu, double lam, double *psi, double *P, double *A,
               int project) {
  *psi = nh_psi(F, d, mu, lam);
  int rc = nh_stress(F, d, mu, lam, P, A);
  if (rc) return rc;
  if (A && project) psd_project(A, d * d);
  return OR_OK;
}

int or_psd_project(double *A, int n) {
  if (n < 1 || n > 9) return OR_E_ARG;
  psd_project(A, n);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Incremental potential, gradient and Hessian-vector product           */
/* (Eq. discrete_energy, Eq. F_update, Sec. 2.2.5)                      */
/* ------------------------------------------------------------------ */

/* Per-particle kinematics fixed for one implicit solve: the stencil nodes,
 * N_ip and c_ip = F_p^nT grad N_ip(x_p^n), so that
 * F_p(u) = (I + sum_i u_i grad N_ip^T) F_p^n = F_p^n + sum_i u_i c_ip^T. */
typedef struct {
  int ss, d;
  int *node;   /* [np][ss] */
  double *N;   /* [np][ss] */
  double *c;   /* [np][ss][d] */
} kin;

static void kin_free(kin *K) {
  free(K->node);
  free(K->N);
  free(K->c);
}

static int kin_build(const or_domain *D, kin *K) {
  const int d = D->dim, ss = stencil_size(D);
  K->ss = ss;
  K->d = d;
  size_t np = (size_t)(D->np > 0 ? D->np : 1);
  K->node = (int *)malloc(sizeof(int) * np * ss);
  K->N = (double *)malloc(sizeof(double) * np * ss);
  K->c = (double *)malloc(sizeof(double) * np * ss * d);
  if (!K->node || !K->N || !K->c) {
    kin_free(K);
    return OR_E_NOMEM;
  }
  for (int p = 0; p < D->np; ++p) {
    stencil st;
    if (stencil_at(D, &D->x[p * d], &st)) {
      kin_free(K);
      return OR_E_OUT_OF_GRID;
    }
    const double *Fn = &D->F[p * d * d];
    for (int s = 0; s < ss; ++s) {
      int i;
      double N, gN[3], dxv[3];
      stencil_node(D, &st, s, &i, &N, gN, dxv);
      K->node[p * ss + s] = i;
      K->N[p * ss + s] = N;
      for (int b = 0; b < d; ++b) {
        double cb = 0.0;
        for (int e = 0; e < d; ++e) cb += Fn[e * d + b] * gN[e];
        K->c[(p * ss + s) * d + b] = cb;
      }
    }
  }
  return OR_OK;
}

/* F_p(u) = F_p^n + sum_i u_i c_ip^T */
static void particle_F(const or_domain *D, const kin *K, int p, const double *u, double *F) {
  const int d = D->dim, ss = K->ss;
  for (int k = 0; k < d * d; ++k) F[k] = D->F[p * d * d + k];
  for (int s = 0; s < ss; ++s) {
    const int i = K->node[p * ss + s];
    const double *c = &K->c[(p * ss + s) * d];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) F[a * d + b] += u[i * d + a] * c[b];
  }
}

static int is_active(const or_domain *D, int i) { return D->m[i] > 0.0; }

/* E(u) = sum_i m_i/(2 dt^2) |u_i - dt v_i^n|^2 + sum_p V_p Psi(F_p(u)) - sum_i m_i g.u_i
 * (Eq. discrete_energy with x_hat = x^n + u, x_tilde = x^n + dt v^n and
 * f_ext = m_i g; the constant -sum x_i^n . f_ext is dropped). */
static double energy_k(const or_domain *D, const kin *K, double dt, const double *grav,
                       const double *u) {
  const int d = D->dim, nn = nnodes(D);
  double E = 0.0;
  for (int i = 0; i < nn; ++i) {
    if (!is_active(D, i)) continue;
    double s2 = 0.0, gu = 0.0;
    for (int a = 0; a < d; ++a) {
      const double r = u[i * d + a] - dt * D->vn[i * d + a];
      s2 += r * r;
      gu += grav[a] * u[i * d + a];
    }
    E += D->m[i] / (2.0 * dt * dt) * s2 - D->m[i] * gu;
  }
  for (int p = 0; p < D->np; ++p) {
    double F[9];
    particle_F(D, K, p, u, F);
    const int mt = D->mat[p];
    E += D->vol[p] * nh_psi(F, d, D->mu[mt], D->lam[mt]);
  }
  return E;
}

/* grad E: m_i/dt^2 (u_i - dt v_i) - m_i g + sum_p V_p P(F_p) c_ip  on every
 * active node (the negative of the residual of Eq. grid_residual). */
static int gradient_k(const or_domain *D, const kin *K, double dt, const double *grav,
                      const double *u, double *g) {
  const int d = D->dim, nn = nnodes(D), ss = K->ss;
  for (int i = 0; i < nn * d; ++i) g[i] = 0.0;
  for (int p = 0; p < D->np; ++p) {
    double F[9], P[9];
    particle_F(D, K, p, u, F);
    const int mt = D->mat[p];
    if (nh_stress(F, d, D->mu[mt], D->lam[mt], P, NULL)) return OR_E_INVERTED;
    for (int s = 0; s < ss; ++s) {
      const int i = K->node[p * ss + s];
      const double *c = &K->c[(p * ss + s) * d];
      for (int a = 0; a < d; ++a) {
        double t = 0.0;
        for (int b = 0; b < d; ++b) t += P[a * d + b] * c[b];
        g[i * d + a] += D->vol[p] * t;
      }
    }
  }
  for (int i = 0; i < nn; ++i) {
    if (!is_active(D, i)) continue;
    for (int a = 0; a < d; ++a)
      g[i * d + a] += D->m[i] / (dt * dt) * (u[i * d + a] - dt * D->vn[i * d + a]) - D->m[i] * grav[a];
  }
  return OR_OK;
}

/* dP/dF of every particle at u, optionally PSD-projected: A_p, [np][d^4]. */
static int hessian_blocks(const or_domain *D, const kin *K, const double *u, int project,
                          double *A) {
  const int d = D->dim, n = d * d;
  for (int p = 0; p < D->np; ++p) {
    double F[9];
    particle_F(D, K, p, u, F);
    const int mt = D->mat[p];
    double *Ap = &A[(size_t)p * n * n];
    if (nh_stress(F, d, D->mu[mt], D->lam[mt], NULL, Ap)) return OR_E_INVERTED;
    if (project) psd_project(Ap, n);
  }
  return OR_OK;
}

/* (H w)_i = m_i/dt^2 w_i + sum_p V_p (A_p : dF_p) c_ip, dF_p = sum_j w_j c_jp^T
 * (the Hessian of E, Sec. 2.2.5, applied through the particles). */
static void hvp_k(const or_domain *D, const kin *K, const double *A, double dt, const double *w,
                  double *y) {
  const int d = D->dim, nn = nnodes(D), ss = K->ss, n = d * d;
  for (int i = 0; i < nn * d; ++i) y[i] = 0.0;
  for (int p = 0; p < D->np; ++p) {
    double dF[9] = {0};
    for (int s = 0; s < ss; ++s) {
      const int j = K->node[p * ss + s];
      const double *c = &K->c[(p * ss + s) * d];
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) dF[a * d + b] += w[j * d + a] * c[b];
    }
    const double *Ap = &A[(size_t)p * n * n];
    double dP[9];
    for (int r = 0; r < n; ++r) {
      double t = 0.0;
      for (int q = 0; q < n; ++q) t += Ap[r * n + q] * dF[q];
      dP[r] = t;
    }
    for (int s = 0; s < ss; ++s) {
      const int i = K->node[p * ss + s];
      const double *c = &K->c[(p * ss + s) * d];
      for (int a = 0; a < d; ++a) {
        double t = 0.0;
        for (int b = 0; b < d; ++b) t += dP[a * d + b] * c[b];
        y[i * d + a] += D->vol[p] * t;
      }
    }
  }
  for (int i = 0; i < nn; ++i) {
    if (!is_active(D, i)) continue;
    for (int a = 0; a < d; ++a) y[i * d + a] += D->m[i] / (dt * dt) * w[i * d + a];
  }
}

/* Jacobi diagonal of H: m_i/dt^2 + sum_p V_p sum_{b,e} A_(ab),(ae) c_b c_e. */
static void diag_k(const or_domain *D, const kin *K, const double *A, double dt, double *dg) {
  const int d = D->dim, nn = nnodes(D), ss = K->ss, n = d * d;
  for (int i = 0; i < nn * d; ++i) dg[i] = 0.0;
  for (int p = 0; p < D->np; ++p) {
    const double *Ap = &A[(size_t)p * n * n];
    for (int s = 0; s < ss; ++s) {
      const int i = K->node[p * ss + s];
      const double *c = &K->c[(p * ss + s) * d];
      for (int a = 0; a < d; ++a) {
        double t = 0.0;
        for (int b = 0; b < d; ++b)
          for (int e = 0; e < d; ++e) t += Ap[(a * d + b) * n + (a * d + e)] * c[b] * c[e];
        dg[i * d + a] += D->vol[p] * t;
      }
    }
  }
  for (int i = 0; i < nn; ++i) {
    if (!is_active(D, i)) continue;
    for (int a = 0; a < d; ++a) dg[i * d + a] += D->m[i] / (dt * dt);
  }
}

/* E(u + alpha du) - E(u), evaluated term by term in a form free of the
 * cancellation of two large totals (exact arithmetic gives the difference of
 * two energies; this is the comparison of the halving line search, Sec. 2.2.5):
 *   inertia:  m/(2dt^2) (2 alpha r.du + alpha^2 |du|^2), r = u - dt v^n
 *   gravity: -alpha m g.du
 *   elastic:  V [mu/2 (2 F:D + D:D) - mu L + lam/2 L (2 ln J + L)],
 *             D = alpha sum du_i c_i^T, L = log1p(dJ/J),
 *             dJ = det(F+D) - det F expanded in powers of D.
 * Returns +inf when any particle reaches J <= 0. */
static double delta_energy_k(const or_domain *D, const kin *K, double dt, const double *grav,
                             const double *u, const double *du, double alpha) {
  const int d = D->dim, nn = nnodes(D), ss = K->ss;
  double dE = 0.0;
  for (int i = 0; i < nn; ++i) {
    if (!is_active(D, i)) continue;
    double rd = 0.0, dd = 0.0, gd = 0.0;
    for (int a = 0; a < d; ++a) {
      const double r = u[i * d + a] - dt * D->vn[i * d + a];
      rd += r * du[i * d + a];
      dd += du[i * d + a] * du[i * d + a];
      gd += grav[a] * du[i * d + a];
    }
    dE += D->m[i] / (2.0 * dt * dt) * (2.0 * alpha * rd + alpha * alpha * dd) - alpha * D->m[i] * gd;
  }
  for (int p = 0; p < D->np; ++p) {
    double F[9], Dm[9] = {0};
    particle_F(D, K, p, u, F);
    for (int s = 0; s < ss; ++s) {
      const int j = K->node[p * ss + s];
      const double *c = &K->c[(p * ss + s) * d];
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) Dm[a * d + b] += du[j * d + a] * c[b];
    }
    for (int k = 0; k < d * d; ++k) Dm[k] *= alpha;
    const double J = det_d(F, d);
    double CF[9], CD[9];
    cofactor(F, d, CF);
    double dJ = 0.0;
    if (d == 2) {
      for (int k = 0; k < 4; ++k) dJ += CF[k] * Dm[k];
      dJ += det_d(Dm, 2);
    } else {
      cofactor(Dm, 3, CD);
      for (int k = 0; k < 9; ++k) dJ += CF[k] * Dm[k];
      for (int k = 0; k < 9; ++k) dJ += F[k] * CD[k];
      dJ += det_d(Dm, 3);
    }
    if (!(J > 0.0) || !(J + dJ > 0.0)) return INFINITY;
    const double lnJ = log(J);
    const double L = log1p(dJ / J);
    double FD = 0.0, DD = 0.0;
    for (int k = 0; k < d * d; ++k) {
      FD += F[k] * Dm[k];
      DD += Dm[k] * Dm[k];
    }
    const int mt = D->mat[p];
    const double mu = D->mu[mt], lam = D->lam[mt];
    dE += D->vol[p] * (0.5 * mu * (2.0 * FD + DD) - mu * L + 0.5 * lam * L * (2.0 * lnJ + L));
  }
  return dE;
}

/* ------------------------------------------------------------------ */
/* Dirichlet data                                                       */
/* ------------------------------------------------------------------ */

/* Prescribed displacement of DOF (i, a) for scene group g over a step dt.
 * FIX: 0.  TRANSLATE: dt * velocity.  ROTATE: incremental rigid rotation of
 * the node position about an axis (Rodrigues). */
static double scene_value(const or_domain *D, int g, int i, int a, double dt) {
  const double *pr = &D->bc_param[8 * g];
  if (D->bc_kind[g] == BC_FIX) return 0.0;
  if (D->bc_kind[g] == BC_TRANSLATE) return dt * pr[a];
  /* ROTATE: pr = {cx, cy, cz, kx, ky, kz, omega}; 3D only */
  int idx[3];
  double xi[3] = {0, 0, 0};
  node_index(D, i, idx);
  node_pos(D, idx, xi);
  const double th = pr[6] * dt;
  const double r[3] = {xi[0] - pr[0], xi[1] - pr[1], xi[2] - pr[2]};
  const double k[3] = {pr[3], pr[4], pr[5]};
  const double kr = k[0] * r[0] + k[1] * r[1] + k[2] * r[2];
  const double kxr[3] = {k[1] * r[2] - k[2] * r[1], k[2] * r[0] - k[0] * r[2], k[0] * r[1] - k[1] * r[0]};
  const double ct = cos(th), st = sin(th);
  const double rr = r[a] * ct + kxr[a] * st + k[a] * kr * (1.0 - ct);
  return rr - r[a];
}

/* Dirichlet flags and values of every DOF for a step dt: scene groups first,
 * then the Schwarz receivers (velocity data times dt); only active nodes. */
int or_dirichlet(const or_domain *D, double dt, unsigned char *dir, double *ud) {
  const int d = D->dim, nn = nnodes(D);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < d; ++a) {
      dir[i * d + a] = 0;
      ud[i * d + a] = 0.0;
      if (!is_active(D, i)) continue;
      const int g = D->bcg[i * d + a];
      if (g >= 0) {
        dir[i * d + a] = 1;
        ud[i * d + a] = scene_value(D, g, i, a, dt);
      } else if (D->use_schwarz_bc && D->recv[i]) {
        dir[i * d + a] = 1;
        ud[i * d + a] = dt * D->vbc[i * d + a];
      }
    }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Newton's method with Jacobi-PCG and halving line search (Sec. 2.2.5) */
/* ------------------------------------------------------------------ */

static double dot_masked(const double *a, const double *b, const unsigned char *fr, int n) {
  double s = 0.0;
  for (int k = 0; k < n; ++k)
    if (fr[k]) s += a[k] * b[k];
  return s;
}

/* Minimises E over the free DOFs (active and not Dirichlet).  u^0 = dt v^n on
 * free DOFs and the prescribed values on Dirichlet DOFs.  Stop when
 * |g_free| <= max(rtol |g_free(u^0)|, atol * sum_i m_i * dx / dt^2), tested
 * before the line search (the paper gives no stopping rule; the absolute
 * floor keeps a nearly equilibrated solve from iterating on rounding noise).
 * Direction: PCG from 0 on H d = -g with the Jacobi preconditioner, stop at
 * |r| <= cg_rtol |r_0|.  Line search: alpha = 1, halved while E does not
 * decrease, at most max_ls halvings; failure keeps u and ends the solve. */
/* The solution of an implicit solve kept for the same solve of the next
 * Schwarz iteration (warm start): the displacement u and node masses m of
 * its grid, and its reference gradient norm.  have = 0 until filled. */
typedef struct {
  double *u, *m;
  double gref;
  int have;
} or_warm;

static int solve_from(or_domain *D, double dt, const or_solve_opts *opt, or_solve_stats *st, const or_warm *w);

int or_solve(or_domain *D, double dt, const or_solve_opts *opt, or_solve_stats *st) {
  return solve_from(D, dt, opt, st, NULL);
}

/* or_solve, optionally warm-started: with w filled, a free DOF of a node
 * that was active in w's grid starts from w's displacement instead of
 * dt v^n, and the Newton test is relative to w's reference norm (the
 * initial gradient norm of the cold-started solve of the first Schwarz
 * iteration), so that a start near the solution does not tighten the test. */
static int solve_from(or_domain *D, double dt, const or_solve_opts *opt, or_solve_stats *st, const or_warm *w) {
  const int d = D->dim, nn = nnodes(D), n = d * d, ndof = nn * d;
  memset(st, 0, sizeof(*st));
  kin K;
  int rc = kin_build(D, &K);
  if (rc) return rc;
  unsigned char *dir = (unsigned char *)malloc((size_t)ndof);
  unsigned char *fr = (unsigned char *)malloc((size_t)ndof);
  double *ud = (double *)malloc(sizeof(double) * ndof);
  double *g = (double *)malloc(sizeof(double) * ndof);
  double *dg = (double *)malloc(sizeof(double) * ndof);
  double *del = (double *)malloc(sizeof(double) * ndof);
  double *r = (double *)malloc(sizeof(double) * ndof);
  double *z = (double *)malloc(sizeof(double) * ndof);
  double *pv = (double *)malloc(sizeof(double) * ndof);
  double *q = (double *)malloc(sizeof(double) * ndof);
  double *A = (double *)malloc(sizeof(double) * (size_t)(D->np > 0 ? D->np : 1) * n * n);
  if (!dir || !fr || !ud || !g || !dg || !del || !r || !z || !pv || !q || !A) {
    rc = OR_E_NOMEM;
    goto done;
  }
  or_dirichlet(D, dt, dir, ud);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < d; ++a) {
      const int k = i * d + a;
      fr[k] = (unsigned char)(is_active(D, i) && !dir[k]);
      if (!is_active(D, i))
        D->u[k] = 0.0;
      else if (dir[k])
        D->u[k] = ud[k];
      else if (w && w->have && w->m[i] > 0.0)
        D->u[k] = w->u[k];
      else
        D->u[k] = dt * D->vn[k];
    }
  /* gradient scale of the absolute floor: total node mass * dx / dt^2, the
   * force that displaces the whole domain by one cell in one step */
  double mtot = 0.0;
  for (int i = 0; i < nn; ++i)
    if (is_active(D, i)) mtot += D->m[i];
  const double gscale = mtot * grid_dx(D) / (dt * dt);
  for (int it = 0;; ++it) {
    rc = gradient_k(D, &K, dt, opt->gravity, D->u, g);
    if (rc) goto done;
    const double gn = sqrt(dot_masked(g, g, fr, ndof));
    if (it == 0) st->gnorm0 = (w && w->have) ? w->gref : gn;
    st->gnorm = gn;
    const double tol = fmax(opt->newton_rtol * st->gnorm0, opt->newton_atol * gscale);
    if (gn <= tol) {
      st->converged = 1;
      break;
    }
    if (it == opt->max_newton) break;
    rc = hessian_blocks(D, &K, D->u, opt->project_psd, A);
    if (rc) goto done;
    diag_k(D, &K, A, dt, dg);
    /* PCG on H del = -g */
    for (int k = 0; k < ndof; ++k) {
      del[k] = 0.0;
      r[k] = fr[k] ? -g[k] : 0.0;
      z[k] = fr[k] ? r[k] / dg[k] : 0.0;
      pv[k] = z[k];
    }
    double rz = dot_masked(r, z, fr, ndof);
    const double r0 = sqrt(dot_masked(r, r, fr, ndof));
    for (int k = 0; k < opt->max_cg && r0 > 0.0; ++k) {
      hvp_k(D, &K, A, dt, pv, q);
      for (int j = 0; j < ndof; ++j)
        if (!fr[j]) q[j] = 0.0;
      const double pq = dot_masked(pv, q, fr, ndof);
      if (!(pq > 0.0)) break;
      const double alpha = rz / pq;
      for (int j = 0; j < ndof; ++j) {
        del[j] += alpha * pv[j];
        r[j] -= alpha * q[j];
      }
      st->cg_iters += 1;
      if (sqrt(dot_masked(r, r, fr, ndof)) <= opt->cg_rtol * r0) break;
      for (int j = 0; j < ndof; ++j) z[j] = fr[j] ? r[j] / dg[j] : 0.0;
      const double rz_new = dot_masked(r, z, fr, ndof);
      const double beta = rz_new / rz;
      rz = rz_new;
      for (int j = 0; j < ndof; ++j) pv[j] = z[j] + beta * pv[j];
    }
    /* halving line search */
    double alpha = 1.0;
    int accepted = 0;
    for (int ls = 0; ls <= opt->max_ls; ++ls) {
      const double dE = delta_energy_k(D, &K, dt, opt->gravity, D->u, del, alpha);
      if (dE < 0.0) {
        accepted = 1;
        break;
      }
      if (ls == opt->max_ls) break;
      alpha *= 0.5;
      st->ls_halvings += 1;
    }
    if (!accepted) {
      st->ls_failed = 1;
      break;
    }
    for (int j = 0; j < ndof; ++j) D->u[j] += alpha * del[j];
    st->newton_iters += 1;
  }
  st->energy = energy_k(D, &K, dt, opt->gravity, D->u);
  rc = OR_OK;
done:
  kin_free(&K);
  free(dir);
  free(fr);
  free(ud);
  free(g);
  free(dg);
  free(del);
  free(r);
  free(z);
  free(pv);
  free(q);
  free(A);
  return rc;
}

/* Exported single pieces, for the finite-difference pins. */
int or_energy(const or_domain *D, double dt, const double *grav, const double *u, double *E) {
  kin K;
  int rc = kin_build(D, &K);
  if (rc) return rc;
  *E = energy_k(D, &K, dt, grav, u);
  kin_free(&K);
  return OR_OK;
}

int or_delta_energy(const or_domain *D, double dt, const double *grav, const double *u,
                    const double *du, double alpha, double *dE) {
  kin K;
  int rc = kin_build(D, &K);
  if (rc) return rc;
  *dE = delta_energy_k(D, &K, dt, grav, u, du, alpha);
  kin_free(&K);
  return OR_OK;
}

int or_gradient(const or_domain *D, double dt, const double *grav, const double *u, double *g) {
  kin K;
  int rc = kin_build(D, &K);
  if (rc) return rc;
  rc = gradient_k(D, &K, dt, grav, u, g);
  kin_free(&K);
  return rc;
}

int or_hvp(const or_domain *D, double dt, const double *u, const double *w, int project, double *y,
           double *diag) {
  const int n = D->dim * D->dim;
  kin K;
  int rc = kin_build(D, &K);
  if (rc) return rc;
  double *A = (double *)malloc(sizeof(double) * (size_t)(D->np > 0 ? D->np : 1) * n * n);
  if (!A) {
    kin_free(&K);
    return OR_E_NOMEM;
  }
  rc = hessian_blocks(D, &K, u, project, A);
  if (!rc) {
    if (y) hvp_k(D, &K, A, dt, w, y);
    if (diag) diag_k(D, &K, A, dt, diag);
  }
  free(A);
  kin_free(&K);
  return rc;
}

/* ------------------------------------------------------------------ */
/* APIC grid-to-particle, F update, advection (Eqs. g2p_v, g2p_B,       */
/* F_update, advection; Eqs. g2p_v_substep .. advect_substep)           */
/* ------------------------------------------------------------------ */

/* With v_i = u_i / dt on the active nodes:
 *   v_p = sum N_ip v_i,  B_p = sum N_ip v_i (x_i - x_p)^T,
 *   F_p <- (I + sum u_i grad N_ip^T) F_p,  x_p <- x_p + dt v_p. */
/* ------------------------------------------------------------------ */
/* Elastoplastic extension (von Mises, Hencky strain)                   */
/* ------------------------------------------------------------------ */
/* The paper keeps to elasticity and names elastoplastic hinges as future
 * work (Sec. 4.4, Sec. 5).  Reading used here: multiplicative split
 * F = F^E F^P, with the particle storing F^E; the implicit solve sees only
 * the elastic energy Psi(F^E); after G2P's deformation-gradient update the
 * trial F^E is projected onto the von Mises set in logarithmic strain,
 * |dev eps| <= tau_y / (2 mu) with eps = log of the principal stretches
 * (the closest point in eps, which keeps the principal directions and
 * tr eps, hence det F^E).  A material with tau_y <= 0 or infinite is
 * elastic. */

/* Eigen-decomposition of the symmetric d x d matrix C (d = 2, 3) by cyclic
 * Jacobi rotations: C = V diag(w) V^T, V column-major in V[a * d + k]
 * (component a of eigenvector k). */
static void sym_eig_small(const double *C, int d, double *w, double *V) {
  double A[9];
  memcpy(A, C, sizeof(double) * (size_t)(d * d));
  for (int a = 0; a < d; ++a)
    for (int k = 0; k < d; ++k) V[a * d + k] = (a == k) ? 1.0 : 0.0;
  double scale = 0.0;
  for (int k = 0; k < d * d; ++k) scale += A[k] * A[k];
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j) off += A[i * d + j] * A[i * d + j];
    if (off == 0.0 || off <= 1e-34 * scale) break;
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j) {
        const double aij = A[i * d + j];
        if (aij == 0.0) continue;
        /* rotation in the (i, j) plane that zeroes A_ij */
        const double th = (A[j * d + j] - A[i * d + i]) / (2.0 * aij);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < d; ++k) {
          const double aki = A[k * d + i], akj = A[k * d + j];
          A[k * d + i] = c * aki - sn * akj;
          A[k * d + j] = sn * aki + c * akj;
        }
        for (int k = 0; k < d; ++k) {
          const double aik = A[i * d + k], ajk = A[j * d + k];
          A[i * d + k] = c * aik - sn * ajk;
          A[j * d + k] = sn * aik + c * ajk;
        }
        for (int k = 0; k < d; ++k) {
          const double vki = V[k * d + i], vkj = V[k * d + j];
          V[k * d + i] = c * vki - sn * vkj;
          V[k * d + j] = sn * vki + c * vkj;
        }
      }
  }
  for (int k = 0; k < d; ++k) w[k] = A[k * d + k];
}

/* Projection of F (row-major d x d) onto the von Mises set in Hencky strain
 * (see above).  With C = F^T F = V diag(s^2) V^T and eps_k = ln s_k, the
 * projected stretches are s_k exp(-delta n_k), n = dev eps / |dev eps| and
 * delta = |dev eps| - tau_y / (2 mu), so F <- F V diag(exp(-delta n)) V^T.
 * Returns 1 when F was changed. */
static int vm_return(double *F, int d, double mu, double tau_y) {
  if (!(tau_y > 0.0) || isinf(tau_y) || !(mu > 0.0)) return 0;
  double Cm[9], w[3], V[9];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double t = 0.0;
      for (int k = 0; k < d; ++k) t += F[k * d + a] * F[k * d + b];
      Cm[a * d + b] = t;
    }
  sym_eig_small(Cm, d, w, V);
  double eps[3], mean = 0.0;
  for (int k = 0; k < d; ++k) {
    if (!(w[k] > 0.0)) return 0; /* singular F: left to the solver's det check */
    eps[k] = 0.5 * log(w[k]);
    mean += eps[k];
  }
  mean /= d;
  double nd = 0.0, dev[3];
  for (int k = 0; k < d; ++k) {
    dev[k] = eps[k] - mean;
    nd += dev[k] * dev[k];
  }
  nd = sqrt(nd);
  const double ky = tau_y / (2.0 * mu);
  if (nd <= ky) return 0;
  const double delta = nd - ky;
  double f[3];
  for (int k = 0; k < d; ++k) f[k] = exp(-delta * dev[k] / nd);
  /* S = V diag(f) V^T, F <- F S */
  double S[9], Fo[9];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double t = 0.0;
      for (int k = 0; k < d; ++k) t += V[a * d + k] * f[k] * V[b * d + k];
      S[a * d + b] = t;
    }
  memcpy(Fo, F, sizeof(double) * (size_t)(d * d));
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double t = 0.0;
      for (int k = 0; k < d; ++k) t += Fo[a * d + k] * S[k * d + b];
      F[a * d + b] = t;
    }
  return 1;
}

/* 1 when some material of D yields (the reverse mode has no derivative of
 * the projection and refuses such domains). */
static int is_plastic(const or_domain *D) {
  if (!D->tau_y) return 0;
  for (int k = 0; k < D->n_mat; ++k)
    if (D->tau_y[k] > 0.0 && !isinf(D->tau_y[k])) return 1;
  return 0;
}

/* Exported for the plasticity pins. */
int or_vm_return(int d, double *F, double mu, double tau_y) {
  if (d < 2 || d > 3) return -1;
  return vm_return(F, d, mu, tau_y);
}

int or_g2p(or_domain *D, double dt) {
  const int d = D->dim, ss = stencil_size(D);
  for (int p = 0; p < D->np; ++p) {
    stencil st;
    if (stencil_at(D, &D->x[p * d], &st)) return OR_E_OUT_OF_GRID;
    double vp[3] = {0, 0, 0}, Bp[9] = {0}, G[9] = {0};
    for (int s = 0; s < ss; ++s) {
      int i;
      double N, gN[3], dxv[3];
      stencil_node(D, &st, s, &i, &N, gN, dxv);
      if (!is_active(D, i)) continue;
      for (int a = 0; a < d; ++a) {
        const double vi = D->u[i * d + a] / dt;
        vp[a] += N * vi;
        for (int b = 0; b < d; ++b) {
          Bp[a * d + b] += N * vi * dxv[b];
          G[a * d + b] += D->u[i * d + a] * gN[b];
        }
      }
    }
    double *Fp = &D->F[p * d * d];
    double Fnew[9];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double t = Fp[a * d + b];
        for (int e = 0; e < d; ++e) t += G[a * d + e] * Fp[e * d + b];
        Fnew[a * d + b] = t;
      }
    if (D->tau_y) {
      const int mt = D->mat[p];
      vm_return(Fnew, d, D->mu[mt], D->tau_y[mt]);
    }
    for (int k = 0; k < d * d; ++k) {
      Fp[k] = Fnew[k];
      D->B[p * d * d + k] = Bp[k];
    }
    for (int a = 0; a < d; ++a) {
      D->v[p * d + a] = vp[a];
      D->x[p * d + a] += dt * vp[a];
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Interface operators (Sec. 3.2)                                       */
/* ------------------------------------------------------------------ */

/* Gamma_alpha = {i : sum_{p in boundary layer} m_p N_ip > tau} with the sum
 * in fixed point (Eq. boundary_grid_set). */
static int boundary_set(or_domain *D) {
  const int d = D->dim, nn = nnodes(D), ss = stencil_size(D);
  const double scale = fixed_scale(D);
  const long long tau_q = llrint(D->tau * scale);
  for (int i = 0; i < nn; ++i) D->q_bnd[i] = 0;
  for (int p = 0; p < D->np; ++p) {
    if (!(D->flags[p] & 1u)) continue;
    stencil st;
    if (stencil_at(D, &D->x[p * d], &st)) return OR_E_OUT_OF_GRID;
    const double mq = D->mass[p] * scale;
    for (int s = 0; s < ss; ++s) {
      int i;
      double N, gN[3], dxv[3];
      stencil_node(D, &st, s, &i, &N, gN, dxv);
      D->q_bnd[i] += fixed_mass(N, mq);
    }
  }
  for (int i = 0; i < nn; ++i) {
    D->gamma[i] = (unsigned char)(D->q_bnd[i] > tau_q && is_active(D, i));
    D->recv[i] = D->gamma[i];
  }
  return OR_OK;
}

/* Boundary sets of both domains and the overlap arbitration (Eq.
 * overlap_donor): a coarse node and a fine node at the same lattice point,
 * both in their boundary sets, are ambiguous; the side with the larger
 * fixed-point node mass is the donor (ties: the coarse side) and is removed
 * from its own receiver set. */
static int arbitrate(or_domain *B, or_domain *S, int *n_amb);

int or_interface(or_domain *B, or_domain *S, int *n_amb) {
  if (B->dim != S->dim || B->m_ref != S->m_ref || B->h0 != S->h0) return OR_E_ARG;
  int rc = boundary_set(B);
  if (rc) return rc;
  rc = boundary_set(S);
  if (rc) return rc;
  return arbitrate(B, S, n_amb);
}

/* The arbitration of or_interface on boundary sets already built. */
static int arbitrate(or_domain *B, or_domain *S, int *n_amb) {
  const int d = B->dim, nnB = nnodes(B);
  int amb = 0;
  for (int I = 0; I < nnB; ++I) {
    if (!B->gamma[I]) continue;
    int iB[3], jS[3] = {0, 0, 0};
    node_index(B, I, iB);
    int hit = 1;
    for (int a = 0; a < d; ++a) {
      const long long L = B->origin_q[a] + (long long)iB[a] * B->dx_q;
      const long long t = L - S->origin_q[a];
      if (t < 0 || t % S->dx_q != 0 || t / S->dx_q >= S->n[a]) {
        hit = 0;
        break;
      }
      jS[a] = (int)(t / S->dx_q);
    }
    if (!hit) continue;
    const int j = node_flat(S, jS);
    if (!S->gamma[j]) continue;
    amb += 1;
    if (B->q_all[I] >= S->q_all[j])
      B->recv[I] = 0; /* coarse side donates */
    else
      S->recv[j] = 0; /* fine side donates */
  }
  *n_amb = amb;
  return OR_OK;
}

/* Pi_{S->B} (Eq. spatial_projection) on the coarse receivers: every active
 * fine node j is a point mass m_S,j at x_S,j; v_B,I = sum m_j v_j N_I(x_j) /
 * (sum m_j N_I(x_j) + eps_tol).  Non-receivers get 0. */
static int project_sums(const or_domain *S, const or_domain *B, const double *vS, double *num, double *den);

int or_project(const or_domain *S, const or_domain *B, double eps_tol, const double *vS,
               double *out) {
  const int d = B->dim, nnB = nnodes(B);
  double *num = (double *)calloc((size_t)nnB * d, sizeof(double));
  double *den = (double *)calloc((size_t)nnB, sizeof(double));
  if (!num || !den) {
    free(num);
    free(den);
    return OR_E_NOMEM;
  }
  const int rc = project_sums(S, B, vS, num, den);
  if (!rc)
    for (int I = 0; I < nnB; ++I)
      for (int a = 0; a < d; ++a)
        out[I * d + a] = B->recv[I] ? num[I * d + a] / (den[I] + eps_tol) : 0.0;
  free(num);
  free(den);
  return rc;
}

/* The sums of Pi_{S->B}: num_I += sum_j m_j N_I(x_j) v_j, den_I += sum_j
 * m_j N_I(x_j) over the active fine nodes j. */
static int project_sums(const or_domain *S, const or_domain *B, const double *vS, double *num, double *den) {
  const int d = B->dim, nnS = nnodes(S), ss = stencil_size(B);
  for (int j = 0; j < nnS; ++j) {
    if (!(S->m[j] > 0.0)) continue;
    int jS[3];
    double xj[3] = {0, 0, 0};
    node_index(S, j, jS);
    node_pos(S, jS, xj);
    stencil st;
    if (stencil_at(B, xj, &st)) return OR_E_OUT_OF_GRID;
    for (int s = 0; s < ss; ++s) {
      int I;
      double N, gN[3], dxv[3];
      stencil_node(B, &st, s, &I, &N, gN, dxv);
      const double w = S->m[j] * N;
      den[I] += w;
      for (int a = 0; a < d; ++a) num[I * d + a] += w * vS[j * d + a];
    }
  }
  return OR_OK;
}

/* I_{B->S} (Eq. interp_BtoS) on the fine receivers: v_S,j = sum_I v_B,I
 * N_I(x_S,j), inactive coarse nodes carrying zero velocity.  Non-receivers
 * get 0. */
int or_interp(const or_domain *B, const double *vB, const or_domain *S, double *out) {
  const int d = B->dim, nnS = nnodes(S), ss = stencil_size(B);
  for (int j = 0; j < nnS; ++j) {
    for (int a = 0; a < d; ++a) out[j * d + a] = 0.0;
    if (!S->recv[j]) continue;
    int jS[3];
    double xj[3] = {0, 0, 0};
    node_index(S, j, jS);
    node_pos(S, jS, xj);
    stencil st;
    if (stencil_at(B, xj, &st)) return OR_E_OUT_OF_GRID;
    for (int s = 0; s < ss; ++s) {
      int I;
      double N, gN[3], dxv[3];
      stencil_node(B, &st, s, &I, &N, gN, dxv);
      if (!(B->m[I] > 0.0)) continue;
      for (int a = 0; a < d; ++a) out[j * d + a] += N * vB[I * d + a];
    }
  }
  return OR_OK;
}

/* T_m (Eq. temporal_interp): (1 - m/M) v^n + (m/M) v^{n+1}. */
void or_temporal(int n, int m, int M, const double *vn, const double *vn1, double *out) {
  const double a = (double)m / (double)M;
  for (int k = 0; k < n; ++k) out[k] = (1.0 - a) * vn[k] + a * vn1[k];
}

/* ------------------------------------------------------------------ */
/* Frames                                                               */
/* ------------------------------------------------------------------ */

static double norm_diff_masked(const double *a, const double *b, const unsigned char *mask, int nn,
                               int d, double *norm_a) {
  double s = 0.0, t = 0.0;
  for (int i = 0; i < nn; ++i) {
    if (!mask[i]) continue;
    for (int c = 0; c < d; ++c) {
      const double e = a[i * d + c] - b[i * d + c];
      s += e * e;
      t += a[i * d + c] * a[i * d + c];
    }
  }
  *norm_a = sqrt(t);
  return sqrt(s);
}

/* One backward-Euler step of a single domain (Sec. 2.2): P2G, implicit
 * solve, G2P with F update and advection. */
int or_single_frame(or_domain *D, double dt, const or_solve_opts *opt, or_solve_stats *st) {
  int rc = or_p2g(D);
  if (rc) return rc;
  D->use_schwarz_bc = 0;
  rc = or_solve(D, dt, opt, st);
  if (rc) return rc;
  return or_g2p(D, dt);
}

/* Warm-start slots of domain D (one per implicit solve of a Schwarz
 * iteration), or NULL when out of memory. */
static or_warm *warm_alloc(const or_domain *D, int n_slots) {
  or_warm *w = (or_warm *)calloc((size_t)n_slots, sizeof(or_warm));
  if (!w) return NULL;
  const int nn = nnodes(D);
  for (int j = 0; j < n_slots; ++j) {
    w[j].u = (double *)malloc(sizeof(double) * nn * D->dim);
    w[j].m = (double *)malloc(sizeof(double) * nn);
    if (!w[j].u || !w[j].m) {
      for (int q = 0; q <= j; ++q) {
        free(w[q].u);
        free(w[q].m);
      }
      free(w);
      return NULL;
    }
  }
  return w;
}

static void warm_free(or_warm *w, int n_slots) {
  if (!w) return;
  for (int j = 0; j < n_slots; ++j) {
    free(w[j].u);
    free(w[j].m);
  }
  free(w);
}

/* Keeps a solve's solution and grid masses for the next iteration; the
 * reference norm is that of the first (cold-started) solve. */
static void warm_keep(or_warm *w, const or_domain *D, const or_solve_stats *ss) {
  const int nn = nnodes(D);
  memcpy(w->u, D->u, sizeof(double) * nn * D->dim);
  memcpy(w->m, D->m, sizeof(double) * nn);
  if (!w->have) w->gref = ss->gnorm0;
  w->have = 1;
}

/* One global frame t_n -> t_{n+1} of the multiplicative Schwarz method
 * (Alg. 1, Secs. 3.3-3.5).  Readings where the paper is open:
 *  - Pi reads the latest fine P2G grid (Step 0 at k = 0, the grid after the
 *    last sub-step otherwise); the projected data computed for the residual
 *    of iteration k is the coarse boundary data of iteration k+1;
 *  - v_GS^(0) = I(v_B^n) (Step 0, "previous time step" velocity);
 *  - residual denominators are floored at 1e-30, an empty receiver set gives
 *    r = 0, and the frame ends after k_max iterations if not converged. */
int or_schwarz_frame(or_domain *B, or_domain *S, double dT, const or_schwarz_opts *o,
                     or_schwarz_stats *st) {
  const int d = B->dim, nnB = nnodes(B), nnS = nnodes(S), npS = S->np;
  const double dt = dT / (double)o->M;
  int rc = OR_OK;
  memset(st, 0, sizeof(*st));
  double *sx = (double *)malloc(sizeof(double) * (size_t)(npS > 0 ? npS : 1) * d);
  double *sv = (double *)malloc(sizeof(double) * (size_t)(npS > 0 ? npS : 1) * d);
  double *sB = (double *)malloc(sizeof(double) * (size_t)(npS > 0 ? npS : 1) * d * d);
  double *sF = (double *)malloc(sizeof(double) * (size_t)(npS > 0 ? npS : 1) * d * d);
  double *vBn = (double *)malloc(sizeof(double) * nnB * d);
  double *vBk = (double *)malloc(sizeof(double) * nnB * d);
  double *vGB = (double *)malloc(sizeof(double) * nnB * d);
  double *vGBnew = (double *)malloc(sizeof(double) * nnB * d);
  double *vGSprev = (double *)malloc(sizeof(double) * nnS * d);
  double *vGSn = (double *)malloc(sizeof(double) * nnS * d);
  double *vGSn1 = (double *)malloc(sizeof(double) * nnS * d);
  or_warm *wB = NULL, *wS = NULL;
  if (!sx || !sv || !sB || !sF || !vBn || !vBk || !vGB || !vGBnew || !vGSprev || !vGSn || !vGSn1) {
    rc = OR_E_NOMEM;
    goto done;
  }
  /* Frame start: the fine state is stored (Eq. store_states), both grids are
   * built and the interface sets formed. */
  memcpy(sx, S->x, sizeof(double) * npS * d);
  memcpy(sv, S->v, sizeof(double) * npS * d);
  memcpy(sB, S->B, sizeof(double) * npS * d * d);
  memcpy(sF, S->F, sizeof(double) * npS * d * d);
  if ((rc = or_p2g(B)) || (rc = or_p2g(S))) goto done;
  if ((rc = or_interface(B, S, &st->n_amb))) goto done;
  for (int i = 0; i < nnB; ++i) st->n_recv_B += B->recv[i];
  for (int i = 0; i < nnS; ++i) st->n_recv_S += S->recv[i];
  memcpy(vBn, B->vn, sizeof(double) * nnB * d);
  if ((rc = or_project(S, B, o->eps_tol, S->vn, vGB))) goto done;
  if ((rc = or_interp(B, vBn, S, vGSprev))) goto done;
  if (o->warm_start && (!(wB = warm_alloc(B, 1)) || !(wS = warm_alloc(S, o->M)))) {
    rc = OR_E_NOMEM;
    goto done;
  }
  for (int k = 0; k < (o->force_iters > 0 ? o->force_iters : o->k_max); ++k) {
    or_solve_stats ss;
    /* the coarse solve over dT with the projected data on its receivers */
    memcpy(B->vbc, vGB, sizeof(double) * nnB * d);
    B->use_schwarz_bc = 1;
    if ((rc = solve_from(B, dT, &o->coarse, &ss, wB))) goto done;
    if (wB) warm_keep(wB, B, &ss);
    st->newton_B += ss.newton_iters;
    st->cg_B += ss.cg_iters;
    st->ls_B += ss.ls_halvings;
    st->unconv_B += !ss.converged;
    st->lsfail_B += ss.ls_failed;
    for (int i = 0; i < nnB; ++i)
      for (int a = 0; a < d; ++a) vBk[i * d + a] = (B->m[i] > 0.0) ? B->u[i * d + a] / dT : 0.0;
    /* the fine domain restarts from the stored state: M sub-steps driven by
     * the temporal interpolation of the two coarse endpoints */
    memcpy(S->x, sx, sizeof(double) * npS * d);
    memcpy(S->v, sv, sizeof(double) * npS * d);
    memcpy(S->B, sB, sizeof(double) * npS * d * d);
    memcpy(S->F, sF, sizeof(double) * npS * d * d);
    if ((rc = or_p2g(S))) goto done;
    if ((rc = or_interp(B, vBn, S, vGSn))) goto done;
    if ((rc = or_interp(B, vBk, S, vGSn1))) goto done;
    for (int m = 1; m <= o->M; ++m) {
      or_temporal(nnS * d, m, o->M, vGSn, vGSn1, S->vbc);
      S->use_schwarz_bc = 1;
      if ((rc = solve_from(S, dt, &o->fine, &ss, wS ? &wS[m - 1] : NULL))) goto done;
      if (wS) warm_keep(&wS[m - 1], S, &ss);
      st->newton_S += ss.newton_iters;
      st->cg_S += ss.cg_iters;
      st->ls_S += ss.ls_halvings;
      st->unconv_S += !ss.converged;
      st->lsfail_S += ss.ls_failed;
      if ((rc = or_g2p(S, dt))) goto done;
      if ((rc = or_p2g(S))) goto done;
    }
    /* projection for the next iteration and the interface changes (Eqs.
     * convergence_residuals, convergence_criterion) */
    if ((rc = or_project(S, B, o->eps_tol, S->vn, vGBnew))) goto done;
    double nB, nS;
    const double dB = norm_diff_masked(vGBnew, vGB, B->recv, nnB, d, &nB);
    const double dS = norm_diff_masked(vGSn1, vGSprev, S->recv, nnS, d, &nS);
    st->r_B = dB / fmax(nB, 1e-30);
    st->r_S = dS / fmax(nS, 1e-30);
    memcpy(vGB, vGBnew, sizeof(double) * nnB * d);
    memcpy(vGSprev, vGSn1, sizeof(double) * nnS * d);
    st->iters = k + 1;
    if (o->force_iters > 0) {
      st->converged = st->r_B <= o->eps_conv && st->r_S <= o->eps_conv;
      if (k + 1 == o->force_iters) break;
      continue;
    }
    if (st->r_B <= o->eps_conv && st->r_S <= o->eps_conv) {
      st->converged = 1;
      break;
    }
  }
  /* the coarse particles move with the last coarse solution (Sec. 3.5) */
  rc = or_g2p(B, dT);
done:
  free(sx);
  free(sv);
  free(sB);
  free(sF);
  free(vBn);
  free(vBk);
  free(vGB);
  free(vGBnew);
  free(vGSprev);
  free(vGSn);
  free(vGSn1);
  warm_free(wB, 1);
  warm_free(wS, o->M);
  return rc;
}

/* Node of G at the lattice point of node i of A, or -1 when G has none. */
static int coincident_node(const or_domain *A, int i, const or_domain *G) {
  int ia[3], jg[3] = {0, 0, 0};
  node_index(A, i, ia);
  for (int a = 0; a < A->dim; ++a) {
    const long long L = A->origin_q[a] + (long long)ia[a] * A->dx_q;
    const long long t = L - G->origin_q[a];
    if (t < 0 || t % G->dx_q != 0 || t / G->dx_q >= G->n[a]) return -1;
    jg[a] = (int)(t / G->dx_q);
  }
  return node_flat(G, jg);
}

/* Fine-fine links of a multi-domain frame.  Arbitration between fine
 * domains (Eq. overlap_donor generalised pairwise): a node in the boundary
 * sets of fine domains f and g at the same lattice point is ambiguous; the
 * side with the larger fixed-point node mass donates (ties: the lower
 * index) and leaves its own receiver set.  Then every remaining receiver
 * node j of f that lies in the material of another fine domain (the
 * coincident node active with a fixed-point mass above that domain's
 * selection threshold) takes its data from the one of largest mass (ties:
 * the lower index): link_g[f][j] = g, link_n[f][j] = its node; -1 where the
 * coarse domain donates.  Returns the number of linked nodes. */
static int fine_links(or_domain **S, int k, int **link_g, int **link_n, int *n_amb) {
  int links = 0;
  for (int f = 0; f < k; ++f) {
    const int nn = nnodes(S[f]);
    for (int j = 0; j < nn; ++j) {
      if (!S[f]->gamma[j]) continue;
      int donor = 0;
      for (int g = 0; g < k; ++g) {
        if (g == f) continue;
        const int jg = coincident_node(S[f], j, S[g]);
        if (jg < 0 || !S[g]->gamma[jg]) continue;
        if (f < g) *n_amb += 1;
        const long long qf = S[f]->q_all[j], qg = S[g]->q_all[jg];
        if (qf > qg || (qf == qg && f < g)) donor = 1;
      }
      link_g[f][j] = donor ? -2 : -1; /* -2: leaves the receiver set (below) */
    }
  }
  for (int f = 0; f < k; ++f) {
    const int nn = nnodes(S[f]);
    for (int j = 0; j < nn; ++j) {
      if (link_g[f][j] == -2) S[f]->recv[j] = 0;
      link_g[f][j] = -1;
      link_n[f][j] = -1;
    }
  }
  for (int f = 0; f < k; ++f) {
    const int nn = nnodes(S[f]);
    for (int j = 0; j < nn; ++j) {
      if (!S[f]->recv[j]) continue;
      long long best = 0;
      for (int g = 0; g < k; ++g) {
        if (g == f) continue;
        const int jg = coincident_node(S[f], j, S[g]);
        if (jg < 0 || !(S[g]->m[jg] > 0.0)) continue;
        const long long q = S[g]->q_all[jg];
        if (q <= llrint(S[g]->tau * fixed_scale(S[g]))) continue;
        if (link_g[f][j] < 0 || q > best) {
          link_g[f][j] = g;
          link_n[f][j] = jg;
          best = q;
        }
      }
      if (link_g[f][j] >= 0) links += 1;
    }
  }
  return links;
}

/* Alg. 1 with one coarse domain B and k fine domains S[0..k-1] that overlap
 * B and possibly each other (the several refined regions the conclusion
 * names as future work; readings, since the paper gives no algorithm for
 * them):
 *  - boundary sets as for a pair; each fine domain is arbitrated against B
 *    by the two-domain rule (Eq. overlap_donor), in index order, and fine
 *    domains against each other pairwise (fine_links);
 *  - Pi (Eq. spatial_projection) over the union of the fine point masses:
 *    numerator and denominator summed over all fine domains, then divided on
 *    the coarse receivers;
 *  - each iteration: coarse solve, then every fine domain restored, P2G,
 *    interpolated at both endpoints from the same coarse solution and
 *    sub-cycled.  A fine receiver linked to another fine domain g takes, at
 *    sub-step m, g's grid velocity u/dt of sub-step m of the previous
 *    iteration (fine domains exchange data between iterations, like a block
 *    Jacobi step, so their order does not matter); in the first iteration,
 *    and where g's node was inactive, the coarse data as for the others;
 *  - r_B over the coarse receivers; r_S over the receivers of all fine
 *    domains together, where a linked receiver's datum is its donor's
 *    end-of-frame velocity u/dt of sub-step M (Eqs. convergence_residuals,
 *    convergence_criterion).
 * Fine domains that do not touch each other have no links, and every step
 * is then that of the disjoint case; with k = 1 that of or_schwarz_frame.
 * Statistics sum the fine domains' counts. */
int or_schwarz_frame_multi(or_domain *B, or_domain **S, int k, double dT, const or_schwarz_opts *o,
                           or_schwarz_stats *st) {
  if (k < 1) return OR_E_ARG;
  for (int f = 0; f < k; ++f)
    if (B->dim != S[f]->dim || B->m_ref != S[f]->m_ref || B->h0 != S[f]->h0) return OR_E_ARG;
  const int d = B->dim, nnB = nnodes(B);
  const double dt = dT / (double)o->M;
  int rc = OR_OK;
  memset(st, 0, sizeof(*st));
  double **sx = (double **)calloc((size_t)k, sizeof(double *)), **sv = (double **)calloc((size_t)k, sizeof(double *));
  double **sB = (double **)calloc((size_t)k, sizeof(double *)), **sF = (double **)calloc((size_t)k, sizeof(double *));
  double **vGSprev = (double **)calloc((size_t)k, sizeof(double *));
  double **vGSn = (double **)calloc((size_t)k, sizeof(double *));
  double **vGSn1 = (double **)calloc((size_t)k, sizeof(double *));
  double *vBn = (double *)malloc(sizeof(double) * nnB * d);
  double *vBk = (double *)malloc(sizeof(double) * nnB * d);
  double *vGB = (double *)malloc(sizeof(double) * nnB * d);
  double *vGBnew = (double *)malloc(sizeof(double) * nnB * d);
  double *num = (double *)malloc(sizeof(double) * nnB * d);
  double *den = (double *)malloc(sizeof(double) * nnB);
  or_warm *wB = NULL, **wS = (or_warm **)calloc((size_t)k, sizeof(or_warm *));
  /* fine-fine links and the sub-step solutions they read (previous and
   * current iteration: [m][node][d] and [m][node] per fine domain) */
  int **link_g = (int **)calloc((size_t)k, sizeof(int *)), **link_n = (int **)calloc((size_t)k, sizeof(int *));
  double **prevU = (double **)calloc((size_t)k, sizeof(double *)), **prevM = (double **)calloc((size_t)k, sizeof(double *));
  double **curU = (double **)calloc((size_t)k, sizeof(double *)), **curM = (double **)calloc((size_t)k, sizeof(double *));
  int n_links = 0, have_prev = 0;
  if (!link_g || !link_n || !prevU || !prevM || !curU || !curM || !wS || !sx || !sv || !sB || !sF || !vGSprev || !vGSn || !vGSn1 || !vBn || !vBk || !vGB || !vGBnew || !num || !den) {
    rc = OR_E_NOMEM;
    goto done;
  }
  for (int f = 0; f < k; ++f) {
    const int np = S[f]->np > 0 ? S[f]->np : 1, nnS = nnodes(S[f]);
    sx[f] = (double *)malloc(sizeof(double) * (size_t)np * d);
    sv[f] = (double *)malloc(sizeof(double) * (size_t)np * d);
    sB[f] = (double *)malloc(sizeof(double) * (size_t)np * d * d);
    sF[f] = (double *)malloc(sizeof(double) * (size_t)np * d * d);
    vGSprev[f] = (double *)malloc(sizeof(double) * nnS * d);
    vGSn[f] = (double *)malloc(sizeof(double) * nnS * d);
    vGSn1[f] = (double *)malloc(sizeof(double) * nnS * d);
    link_g[f] = (int *)malloc(sizeof(int) * nnS);
    link_n[f] = (int *)malloc(sizeof(int) * nnS);
    if (!sx[f] || !sv[f] || !sB[f] || !sF[f] || !vGSprev[f] || !vGSn[f] || !vGSn1[f] || !link_g[f] || !link_n[f]) {
      rc = OR_E_NOMEM;
      goto done;
    }
  }
  /* Frame start: fine states stored, all grids built, boundary sets and
   * arbitration */
  for (int f = 0; f < k; ++f) {
    const or_domain *Sf = S[f];
    memcpy(sx[f], Sf->x, sizeof(double) * Sf->np * d);
    memcpy(sv[f], Sf->v, sizeof(double) * Sf->np * d);
    memcpy(sB[f], Sf->B, sizeof(double) * Sf->np * d * d);
    memcpy(sF[f], Sf->F, sizeof(double) * Sf->np * d * d);
  }
  if ((rc = or_p2g(B))) goto done;
  for (int f = 0; f < k; ++f)
    if ((rc = or_p2g(S[f]))) goto done;
  if ((rc = boundary_set(B))) goto done;
  for (int f = 0; f < k; ++f) {
    int amb = 0;
    if ((rc = boundary_set(S[f])) || (rc = arbitrate(B, S[f], &amb))) goto done;
    st->n_amb += amb;
  }
  n_links = fine_links(S, k, link_g, link_n, &st->n_amb);
  for (int f = 0; f < k && n_links; ++f) {
    const size_t nnS = (size_t)nnodes(S[f]), M = (size_t)o->M;
    prevU[f] = (double *)malloc(sizeof(double) * M * nnS * d);
    prevM[f] = (double *)malloc(sizeof(double) * M * nnS);
    curU[f] = (double *)malloc(sizeof(double) * M * nnS * d);
    curM[f] = (double *)malloc(sizeof(double) * M * nnS);
    if (!prevU[f] || !prevM[f] || !curU[f] || !curM[f]) {
      rc = OR_E_NOMEM;
      goto done;
    }
  }
  for (int i = 0; i < nnB; ++i) st->n_recv_B += B->recv[i];
  for (int f = 0; f < k; ++f)
    for (int i = 0; i < nnodes(S[f]); ++i) st->n_recv_S += S[f]->recv[i];
  memcpy(vBn, B->vn, sizeof(double) * nnB * d);
#define PROJECT_ALL(OUT)                                                          \
  do {                                                                            \
    memset(num, 0, sizeof(double) * nnB * d);                                     \
    memset(den, 0, sizeof(double) * nnB);                                         \
    for (int f = 0; f < k; ++f)                                                   \
      if ((rc = project_sums(S[f], B, S[f]->vn, num, den))) goto done;           \
    for (int I = 0; I < nnB; ++I)                                                 \
      for (int a = 0; a < d; ++a)                                                 \
        (OUT)[I * d + a] = B->recv[I] ? num[I * d + a] / (den[I] + o->eps_tol) : 0.0; \
  } while (0)
  PROJECT_ALL(vGB);
  for (int f = 0; f < k; ++f)
    if ((rc = or_interp(B, vBn, S[f], vGSprev[f]))) goto done;
  if (o->warm_start) {
    if (!(wB = warm_alloc(B, 1))) rc = OR_E_NOMEM;
    for (int f = 0; f < k && !rc; ++f)
      if (!(wS[f] = warm_alloc(S[f], o->M))) rc = OR_E_NOMEM;
    if (rc) goto done;
  }
  for (int it = 0; it < (o->force_iters > 0 ? o->force_iters : o->k_max); ++it) {
    or_solve_stats ss;
    /* the coarse solve with the projected data */
    memcpy(B->vbc, vGB, sizeof(double) * nnB * d);
    B->use_schwarz_bc = 1;
    if ((rc = solve_from(B, dT, &o->coarse, &ss, wB))) goto done;
    if (wB) warm_keep(wB, B, &ss);
    st->newton_B += ss.newton_iters;
    st->cg_B += ss.cg_iters;
    st->ls_B += ss.ls_halvings;
    st->unconv_B += !ss.converged;
    st->lsfail_B += ss.ls_failed;
    for (int i = 0; i < nnB; ++i)
      for (int a = 0; a < d; ++a) vBk[i * d + a] = (B->m[i] > 0.0) ? B->u[i * d + a] / dT : 0.0;
    /* every fine domain restarts from its stored state and is sub-cycled */
    for (int f = 0; f < k; ++f) {
      or_domain *Sf = S[f];
      const int nnS = nnodes(Sf);
      memcpy(Sf->x, sx[f], sizeof(double) * Sf->np * d);
      memcpy(Sf->v, sv[f], sizeof(double) * Sf->np * d);
      memcpy(Sf->B, sB[f], sizeof(double) * Sf->np * d * d);
      memcpy(Sf->F, sF[f], sizeof(double) * Sf->np * d * d);
      if ((rc = or_p2g(Sf))) goto done;
      if ((rc = or_interp(B, vBn, Sf, vGSn[f]))) goto done;
      if ((rc = or_interp(B, vBk, Sf, vGSn1[f]))) goto done;
      for (int m = 1; m <= o->M; ++m) {
        or_temporal(nnS * d, m, o->M, vGSn[f], vGSn1[f], Sf->vbc);
        /* linked receivers: the donor's sub-step-m velocity of the previous
         * iteration, where its node was active */
        for (int j = 0; j < nnS && have_prev; ++j) {
          const int g = link_g[f][j];
          if (g < 0) continue;
          const size_t jg = (size_t)(m - 1) * nnodes(S[g]) + link_n[f][j];
          if (!(prevM[g][jg] > 0.0)) continue;
          for (int a = 0; a < d; ++a) Sf->vbc[j * d + a] = prevU[g][jg * d + a] / dt;
        }
        Sf->use_schwarz_bc = 1;
        if ((rc = solve_from(Sf, dt, &o->fine, &ss, wS[f] ? &wS[f][m - 1] : NULL))) goto done;
        if (wS[f]) warm_keep(&wS[f][m - 1], Sf, &ss);
        if (n_links) {
          memcpy(curU[f] + (size_t)(m - 1) * nnS * d, Sf->u, sizeof(double) * nnS * d);
          memcpy(curM[f] + (size_t)(m - 1) * nnS, Sf->m, sizeof(double) * nnS);
        }
        st->newton_S += ss.newton_iters;
        st->cg_S += ss.cg_iters;
        st->ls_S += ss.ls_halvings;
        st->unconv_S += !ss.converged;
        st->lsfail_S += ss.ls_failed;
        if ((rc = or_g2p(Sf, dt))) goto done;
        if ((rc = or_p2g(Sf))) goto done;
      }
    }
    /* linked receivers' data for the residual: the donor's end-of-frame
     * velocity (sub-step M) of this iteration */
    for (int f = 0; f < k && n_links; ++f)
      for (int j = 0; j < nnodes(S[f]); ++j) {
        const int g = link_g[f][j];
        if (g < 0) continue;
        const size_t jg = (size_t)(o->M - 1) * nnodes(S[g]) + link_n[f][j];
        if (!(curM[g][jg] > 0.0)) continue;
        for (int a = 0; a < d; ++a) vGSn1[f][j * d + a] = curU[g][jg * d + a] / dt;
      }
    if (n_links) {
      for (int f = 0; f < k; ++f) {
        double *t = prevU[f];
        prevU[f] = curU[f];
        curU[f] = t;
        t = prevM[f];
        prevM[f] = curM[f];
        curM[f] = t;
      }
      have_prev = 1;
    }
    /* projection for the next iteration and changes over all interfaces */
    PROJECT_ALL(vGBnew);
    double nB, dB_ = norm_diff_masked(vGBnew, vGB, B->recv, nnB, d, &nB);
    double dS2 = 0.0, nS2 = 0.0;
    for (int f = 0; f < k; ++f) {
      double nSf;
      const double dSf = norm_diff_masked(vGSn1[f], vGSprev[f], S[f]->recv, nnodes(S[f]), d, &nSf);
      dS2 += dSf * dSf;
      nS2 += nSf * nSf;
    }
    st->r_B = dB_ / fmax(nB, 1e-30);
    st->r_S = sqrt(dS2) / fmax(sqrt(nS2), 1e-30);
    memcpy(vGB, vGBnew, sizeof(double) * nnB * d);
    for (int f = 0; f < k; ++f) memcpy(vGSprev[f], vGSn1[f], sizeof(double) * nnodes(S[f]) * d);
    st->iters = it + 1;
    st->converged = st->r_B <= o->eps_conv && st->r_S <= o->eps_conv;
    if (o->force_iters > 0) {
      if (it + 1 == o->force_iters) break;
      continue;
    }
    if (st->converged) break;
  }
#undef PROJECT_ALL
  /* the coarse particles move with the last coarse solution (Sec. 3.5) */
  rc = or_g2p(B, dT);
done:
  for (int f = 0; f < k; ++f) {
    if (sx) free(sx[f]);
    if (sv) free(sv[f]);
    if (sB) free(sB[f]);
    if (sF) free(sF[f]);
    if (vGSprev) free(vGSprev[f]);
    if (vGSn) free(vGSn[f]);
    if (vGSn1) free(vGSn1[f]);
  }
  free(sx);
  free(sv);
  free(sB);
  free(sF);
  free(vGSprev);
  free(vGSn);
  free(vGSn1);
  free(vBn);
  free(vBk);
  free(vGB);
  free(vGBnew);
  free(num);
  free(den);
  for (int f = 0; f < k; ++f) {
    if (link_g) free(link_g[f]);
    if (link_n) free(link_n[f]);
    if (prevU) free(prevU[f]);
    if (prevM) free(prevM[f]);
    if (curU) free(curU[f]);
    if (curM) free(curM[f]);
  }
  free(link_g);
  free(link_n);
  free(prevU);
  free(prevM);
  free(curU);
  free(curM);
  for (int f = 0; f < k && wS; ++f) warm_free(wS[f], o->M);
  free(wS);
  warm_free(wB, 1);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Reverse mode: the adjoint of a frame with respect to the start-of-    */
/* frame particle states and the Lame parameters of every material.      */
/*                                                                      */
/* Discrete decisions (bins, active nodes, boundary and receiver sets,   */
/* the number of Schwarz iterations) are held at their forward values.   */
/* Each implicit solve is differentiated at its minimiser by the         */
/* implicit-function theorem: with g_f(u*; inputs) = 0 on the free DOFs  */
/* and the Dirichlet DOFs fixed by data, the adjoint lambda solves       */
/* H_ff lambda = ubar_f with the Hessian of E at u* (not PSD-projected), */
/* every input receives -lambda^T dg_f/d(input), and the Dirichlet data  */
/* receive ubar_D - (H lambda)_D.  The transfers are transposed exactly, */
/* including the dependence of N_ip and grad N_ip on the particle        */
/* position (second derivatives of the quadratic B-spline).              */
/* ------------------------------------------------------------------ */

/* Second derivatives of N_ip with respect to x_p (d x d, symmetric) at stencil
 * node s: d2w/df2 = (1, -2, 1) per axis for the three stencil offsets. */
static void stencil_hess(const or_domain *D, const stencil *st, int s, double *Hs) {
  const int d = D->dim;
  const double dx = grid_dx(D), i2 = 1.0 / (dx * dx);
  const int k[3] = {s % 3, (s / 3) % 3, s / 9};
  double w[3] = {1, 1, 1}, dw[3] = {0, 0, 0}, ddw[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) {
    w[a] = st->w[a][k[a]];
    dw[a] = st->dw[a][k[a]];
    ddw[a] = (k[a] == 1 ? -2.0 : 1.0) * i2;
  }
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double v = 1.0;
      for (int c = 0; c < d; ++c) {
        if (a == b)
          v *= (c == a) ? ddw[c] : w[c];
        else
          v *= (c == a || c == b) ? dw[c] : w[c];
      }
      Hs[a * d + b] = v;
    }
}

/* A view of a domain with its particle and grid arrays replaced (the
 * forward states stored for the reverse sweep). */
static or_domain view_of(const or_domain *D, double *x, double *v, double *B, double *F, double *m,
                         double *vn, double *u) {
  or_domain V = *D;
  V.x = x;
  V.v = v;
  V.B = B;
  V.F = F;
  V.m = m;
  V.vn = vn;
  V.u = u;
  return V;
}

/* P2G transposed.  Given mbar, vnbar on the nodes (the adjoint of the node
 * mass and of v = (mv)/m), adds the adjoint of x, v, B of the particles. */
static int p2g_adjoint(const or_domain *D, const double *mbar, const double *vnbar, double *xbar,
                       double *vbar, double *Bbar) {
  const int d = D->dim, ss = stencil_size(D);
  const double dx = grid_dx(D), Dinv = 4.0 / (dx * dx);
  for (int p = 0; p < D->np; ++p) {
    stencil st;
    if (stencil_at(D, &D->x[p * d], &st)) return OR_E_OUT_OF_GRID;
    const double mp = D->mass[p];
    const double *vp = &D->v[p * d], *Bp = &D->B[p * d * d];
    for (int s = 0; s < ss; ++s) {
      int i;
      double N, gN[3], dxv[3];
      stencil_node(D, &st, s, &i, &N, gN, dxv);
      const double mi = D->m[i];
      double pb[3] = {0, 0, 0}, mt = mbar[i];
      if (mi > 0.0) {
        for (int a = 0; a < d; ++a) {
          pb[a] = vnbar[i * d + a] / mi;
          mt -= vnbar[i * d + a] * D->vn[i * d + a] / mi;
        }
      }
      double w[3], pw = 0.0;
      for (int a = 0; a < d; ++a) {
        double aff = 0.0;
        for (int b = 0; b < d; ++b) aff += Bp[a * d + b] * dxv[b];
        w[a] = vp[a] + Dinv * aff;
        pw += pb[a] * w[a];
      }
      for (int a = 0; a < d; ++a) {
        vbar[p * d + a] += mp * N * pb[a];
        for (int b = 0; b < d; ++b) Bbar[(p * d + a) * d + b] += mp * N * Dinv * pb[a] * dxv[b];
        double bt = 0.0; /* (B^T pb)_a */
        for (int b = 0; b < d; ++b) bt += Bp[b * d + a] * pb[b];
        xbar[p * d + a] += mp * ((mt + pw) * gN[a] - N * Dinv * bt);
      }
    }
  }
  return OR_OK;
}

/* G2P transposed.  D holds the particle state before G2P and u the grid
 * displacement; given the adjoint of the particle state after G2P (xo, vo,
 * Bo, Fo), adds ubar on the nodes and the adjoint of x and F before G2P
 * (v and B before G2P do not reach the output). */
static int g2p_adjoint(const or_domain *D, double dt, const double *xo, const double *vo,
                       const double *Bo, const double *Fo, double *ubar, double *xbar, double *Fbar) {
  const int d = D->dim, ss = stencil_size(D);
  for (int p = 0; p < D->np; ++p) {
    stencil st;
    if (stencil_at(D, &D->x[p * d], &st)) return OR_E_OUT_OF_GRID;
    const double *Fp = &D->F[p * d * d];
    const double *Fb = &Fo[p * d * d], *Bb = &Bo[p * d * d];
    double vt[3], G[9] = {0};
    for (int a = 0; a < d; ++a) {
      vt[a] = vo[p * d + a] + dt * xo[p * d + a];
      xbar[p * d + a] += xo[p * d + a];
    }
    /* M1 = Fo F^T (for ubar), M2 = F Fo^T (for the position term) */
    double M1[9], M2[9];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double t1 = 0.0, t2 = 0.0;
        for (int c = 0; c < d; ++c) {
          t1 += Fb[a * d + c] * Fp[b * d + c];
          t2 += Fp[a * d + c] * Fb[b * d + c];
        }
        M1[a * d + b] = t1;
        M2[a * d + b] = t2;
      }
    for (int s = 0; s < ss; ++s) {
      int i;
      double N, gN[3], dxv[3], Hs[9];
      stencil_node(D, &st, s, &i, &N, gN, dxv);
      if (!is_active(D, i)) continue;
      stencil_hess(D, &st, s, Hs);
      const double *ui = &D->u[i * d];
      double Bx[3], uv = 0.0, uBx = 0.0, Btu[3], Mu[3];
      for (int a = 0; a < d; ++a) {
        double t = 0.0, t2 = 0.0, t3 = 0.0;
        for (int b = 0; b < d; ++b) {
          t += Bb[a * d + b] * dxv[b];
          t2 += Bb[b * d + a] * ui[b];
          t3 += M2[a * d + b] * ui[b];
        }
        Bx[a] = t;
        Btu[a] = t2;
        Mu[a] = t3;
      }
      for (int a = 0; a < d; ++a) {
        uv += ui[a] * vt[a];
        uBx += ui[a] * Bx[a];
      }
      for (int a = 0; a < d; ++a) {
        double t = 0.0;
        for (int b = 0; b < d; ++b) t += M1[a * d + b] * gN[b];
        ubar[i * d + a] += N * vt[a] / dt + N * Bx[a] / dt + t;
        double h = 0.0;
        for (int b = 0; b < d; ++b) h += Hs[a * d + b] * Mu[b];
        xbar[p * d + a] += (uv / dt + uBx / dt) * gN[a] - N * Btu[a] / dt + h;
      }
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) G[a * d + b] += ui[a] * gN[b];
    }
    /* Fbar_old += (I + G)^T Fo */
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double t = Fb[a * d + b];
        for (int c = 0; c < d; ++c) t += G[c * d + a] * Fb[c * d + b];
        Fbar[p * d * d + a * d + b] += t;
      }
  }
  return OR_OK;
}

/* Adjoint of one converged implicit solve on D (whose u holds the
 * minimiser), see the section comment.  Adds mbar, vnbar (nodes), xbar, Fbar
 * (particles), mubar, lambar (materials) and, where given, vbcbar on the
 * Schwarz receiver DOFs. */
static int solve_adjoint(const or_domain *D, double dt, const double *grav, const double *ubar,
                         double cg_rtol, int max_cg, double *mbar, double *vnbar, double *xbar,
                         double *Fbar, double *mubar, double *lambar, double *vbcbar) {
  const int d = D->dim, nn = nnodes(D), n = d * d, ndof = nn * d, ss = stencil_size(D);
  kin K;
  int rc = kin_build(D, &K);
  if (rc) return rc;
  unsigned char *dir = (unsigned char *)malloc((size_t)ndof);
  unsigned char *fr = (unsigned char *)malloc((size_t)ndof);
  double *ud = (double *)malloc(sizeof(double) * ndof);
  double *lam = (double *)calloc((size_t)ndof, sizeof(double));
  double *r = (double *)malloc(sizeof(double) * ndof);
  double *z = (double *)malloc(sizeof(double) * ndof);
  double *pv = (double *)malloc(sizeof(double) * ndof);
  double *q = (double *)malloc(sizeof(double) * ndof);
  double *dg = (double *)malloc(sizeof(double) * ndof);
  double *A = (double *)malloc(sizeof(double) * (size_t)(D->np > 0 ? D->np : 1) * n * n);
  if (!dir || !fr || !ud || !lam || !r || !z || !pv || !q || !dg || !A) {
    rc = OR_E_NOMEM;
    goto done;
  }
  or_dirichlet(D, dt, dir, ud);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < d; ++a) fr[i * d + a] = (unsigned char)(is_active(D, i) && !dir[i * d + a]);
  if ((rc = hessian_blocks(D, &K, D->u, 0, A))) goto done;
  diag_k(D, &K, A, dt, dg);
  /* PCG on H_ff lambda = ubar_f */
  for (int k = 0; k < ndof; ++k) {
    r[k] = fr[k] ? ubar[k] : 0.0;
    z[k] = fr[k] ? r[k] / dg[k] : 0.0;
    pv[k] = z[k];
  }
  {
    double rz = dot_masked(r, z, fr, ndof);
    const double r0 = sqrt(dot_masked(r, r, fr, ndof));
    for (int k = 0; k < max_cg && r0 > 0.0; ++k) {
      hvp_k(D, &K, A, dt, pv, q);
      for (int j = 0; j < ndof; ++j)
        if (!fr[j]) q[j] = 0.0;
      const double pq = dot_masked(pv, q, fr, ndof);
      if (!(pq > 0.0)) break;
      const double alpha = rz / pq;
      for (int j = 0; j < ndof; ++j) {
        lam[j] += alpha * pv[j];
        r[j] -= alpha * q[j];
      }
      if (sqrt(dot_masked(r, r, fr, ndof)) <= cg_rtol * r0) break;
      for (int j = 0; j < ndof; ++j) z[j] = fr[j] ? r[j] / dg[j] : 0.0;
      const double rz_new = dot_masked(r, z, fr, ndof);
      const double beta = rz_new / rz;
      rz = rz_new;
      for (int j = 0; j < ndof; ++j) pv[j] = z[j] + beta * pv[j];
    }
  }
  /* Dirichlet data: ubar_D - (H lambda)_D, on the Schwarz receiver DOFs */
  if (vbcbar) {
    hvp_k(D, &K, A, dt, lam, q);
    for (int i = 0; i < nn; ++i)
      for (int a = 0; a < d; ++a) {
        const int k = i * d + a;
        if (!is_active(D, i) || !dir[k] || D->bcg[k] >= 0 || !D->use_schwarz_bc || !D->recv[i]) continue;
        vbcbar[k] += dt * (ubar[k] - q[k]);
      }
  }
  /* node inputs: g_i = m_i/dt^2 (u_i - dt v_i) - m_i g + f_int,i */
  for (int i = 0; i < nn; ++i) {
    if (!is_active(D, i)) continue;
    for (int a = 0; a < d; ++a) {
      const int k = i * d + a;
      if (!fr[k]) continue;
      vnbar[k] += lam[k] * D->m[i] / dt;
      mbar[i] -= lam[k] * ((D->u[k] - dt * D->vn[k]) / (dt * dt) - grav[a]);
    }
  }
  /* particle inputs: phi_p = V P(F(u)) : (G_lambda F^n) */
  for (int p = 0; p < D->np; ++p) {
    stencil st;
    if (stencil_at(D, &D->x[p * d], &st)) {
      rc = OR_E_OUT_OF_GRID;
      goto done;
    }
    const double *Fn = &D->F[p * d * d];
    double Gu[9] = {0}, Gl[9] = {0};
    for (int s = 0; s < ss; ++s) {
      int i;
      double N, gN[3], dxv[3];
      stencil_node(D, &st, s, &i, &N, gN, dxv);
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          Gu[a * d + b] += D->u[i * d + a] * gN[b];
          Gl[a * d + b] += lam[i * d + a] * gN[b];
        }
    }
    double H[9], F[9], L[9], P[9], Ap[81];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) H[a * d + b] = (a == b ? 1.0 : 0.0) + Gu[a * d + b];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double t = 0.0, t2 = 0.0;
        for (int c = 0; c < d; ++c) {
          t += H[a * d + c] * Fn[c * d + b];
          t2 += Gl[a * d + c] * Fn[c * d + b];
        }
        F[a * d + b] = t;
        L[a * d + b] = t2;
      }
    const int mt = D->mat[p];
    if (nh_stress(F, d, D->mu[mt], D->lam[mt], P, Ap)) {
      rc = OR_E_INVERTED;
      goto done;
    }
    const double V = D->vol[p];
    /* material: dP/dmu = F - F^-T, dP/dlam = ln J F^-T */
    {
      const double J = det_d(F, d), lnJ = log(J);
      double C[9];
      cofactor(F, d, C); /* F^-T = C / J */
      double smu = 0.0, slam = 0.0;
      for (int k = 0; k < n; ++k) {
        smu += (F[k] - C[k] / J) * L[k];
        slam += lnJ * C[k] / J * L[k];
      }
      mubar[mt] -= V * smu;
      lambar[mt] -= V * slam;
    }
    /* AL = A : L */
    double AL[9];
    for (int r2 = 0; r2 < n; ++r2) {
      double t = 0.0;
      for (int c2 = 0; c2 < n; ++c2) t += Ap[r2 * n + c2] * L[c2];
      AL[r2] = t;
    }
    /* Fbar^n -= V (H^T AL + Gl^T P) */
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double t = 0.0;
        for (int c = 0; c < d; ++c) t += H[c * d + a] * AL[c * d + b] + Gl[c * d + a] * P[c * d + b];
        Fbar[p * d * d + a * d + b] -= V * t;
      }
    /* xbar -= V sum_i Hs_ip (Y1^T u_i + Y2^T lambda_i), Y1 = AL F^nT, Y2 = P F^nT */
    double Y1[9], Y2[9];
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double t1 = 0.0, t2 = 0.0;
        for (int c = 0; c < d; ++c) {
          t1 += AL[a * d + c] * Fn[b * d + c];
          t2 += P[a * d + c] * Fn[b * d + c];
        }
        Y1[a * d + b] = t1;
        Y2[a * d + b] = t2;
      }
    for (int s = 0; s < ss; ++s) {
      int i;
      double N, gN[3], dxv[3], Hs[9];
      stencil_node(D, &st, s, &i, &N, gN, dxv);
      stencil_hess(D, &st, s, Hs);
      double y[3];
      for (int b = 0; b < d; ++b) {
        double t = 0.0;
        for (int a = 0; a < d; ++a) t += Y1[a * d + b] * D->u[i * d + a] + Y2[a * d + b] * lam[i * d + a];
        y[b] = t;
      }
      for (int a = 0; a < d; ++a) {
        double t = 0.0;
        for (int b = 0; b < d; ++b) t += Hs[a * d + b] * y[b];
        xbar[p * d + a] -= V * t;
      }
    }
  }
  rc = OR_OK;
done:
  kin_free(&K);
  free(dir);
  free(fr);
  free(ud);
  free(lam);
  free(r);
  free(z);
  free(pv);
  free(q);
  free(dg);
  free(A);
  return rc;
}

/* Pi_{S->B} transposed: given the adjoint of the projected data on the
 * coarse receivers, adds the adjoint of the fine node masses and velocities
 * (S holds the fine grid the projection read). */
static int project_adjoint(const or_domain *S, const or_domain *B, double eps_tol, const double *pbar,
                           double *mbarS, double *vnbarS) {
  const int d = B->dim, nnB = nnodes(B), nnS = nnodes(S), ss = stencil_size(B);
  double *num = (double *)calloc((size_t)nnB * d, sizeof(double));
  double *den = (double *)calloc((size_t)nnB, sizeof(double));
  if (!num || !den) {
    free(num);
    free(den);
    return OR_E_NOMEM;
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < nnS; ++j) {
      if (!(S->m[j] > 0.0)) continue;
      int jS[3];
      double xj[3] = {0, 0, 0};
      node_index(S, j, jS);
      node_pos(S, jS, xj);
      stencil st;
      if (stencil_at(B, xj, &st)) {
        free(num);
        free(den);
        return OR_E_OUT_OF_GRID;
      }
      for (int s = 0; s < ss; ++s) {
        int I;
        double N, gN[3], dxv[3];
        stencil_node(B, &st, s, &I, &N, gN, dxv);
        if (pass == 0) {
          den[I] += S->m[j] * N;
          for (int a = 0; a < d; ++a) num[I * d + a] += S->m[j] * N * S->vn[j * d + a];
        } else if (B->recv[I]) {
          const double de = den[I] + eps_tol;
          double pn = 0.0;
          for (int a = 0; a < d; ++a) pn += pbar[I * d + a] * num[I * d + a];
          const double denbar = -pn / (de * de);
          double vnum = 0.0;
          for (int a = 0; a < d; ++a) {
            const double numbar = pbar[I * d + a] / de;
            vnbarS[j * d + a] += S->m[j] * N * numbar;
            vnum += S->vn[j * d + a] * numbar;
          }
          mbarS[j] += N * (vnum + denbar);
        }
      }
    }
  }
  free(num);
  free(den);
  return OR_OK;
}

/* I_{B->S} transposed: adds to vBbar the adjoint of the coarse velocity. */
static int interp_adjoint(const or_domain *B, const or_domain *S, const double *ibar, double *vBbar) {
  const int d = B->dim, nnS = nnodes(S), ss = stencil_size(B);
  for (int j = 0; j < nnS; ++j) {
    if (!S->recv[j]) continue;
    int jS[3];
    double xj[3] = {0, 0, 0};
    node_index(S, j, jS);
    node_pos(S, jS, xj);
    stencil st;
    if (stencil_at(B, xj, &st)) return OR_E_OUT_OF_GRID;
    for (int s = 0; s < ss; ++s) {
      int I;
      double N, gN[3], dxv[3];
      stencil_node(B, &st, s, &I, &N, gN, dxv);
      if (!(B->m[I] > 0.0)) continue;
      for (int a = 0; a < d; ++a) vBbar[I * d + a] += N * ibar[j * d + a];
    }
  }
  return OR_OK;
}

/* Adjoint of a particle state: [x d][v d][B d^2][F d^2] per particle block,
 * i.e. four arrays laid out like the state. */
typedef struct {
  double *x, *v, *B, *F;
} adj_state;

static int adj_alloc(adj_state *a, int np, int d) {
  const size_t n = (size_t)(np > 0 ? np : 1);
  a->x = (double *)calloc(n * d, sizeof(double));
  a->v = (double *)calloc(n * d, sizeof(double));
  a->B = (double *)calloc(n * d * d, sizeof(double));
  a->F = (double *)calloc(n * d * d, sizeof(double));
  return (a->x && a->v && a->B && a->F) ? OR_OK : OR_E_NOMEM;
}
static void adj_free(adj_state *a) {
  free(a->x);
  free(a->v);
  free(a->B);
  free(a->F);
}
static void adj_zero(adj_state *a, int np, int d) {
  memset(a->x, 0, sizeof(double) * np * d);
  memset(a->v, 0, sizeof(double) * np * d);
  memset(a->B, 0, sizeof(double) * np * d * d);
  memset(a->F, 0, sizeof(double) * np * d * d);
}

/* Stored forward state of one domain at one point of the frame. */
typedef struct {
  double *x, *v, *B, *F; /* particles */
  double *m, *vn;        /* grid from the P2G of these particles */
  signed char *bcg;      /* scene-BC groups of the DOFs at that P2G */
  double *u, *vbc;       /* solution and Schwarz data of the following solve */
} fwd_point;

static int fwd_alloc(fwd_point *f, const or_domain *D) {
  const int d = D->dim, nn = nnodes(D);
  const size_t np = (size_t)(D->np > 0 ? D->np : 1);
  f->x = (double *)malloc(sizeof(double) * np * d);
  f->v = (double *)malloc(sizeof(double) * np * d);
  f->B = (double *)malloc(sizeof(double) * np * d * d);
  f->F = (double *)malloc(sizeof(double) * np * d * d);
  f->m = (double *)malloc(sizeof(double) * nn);
  f->vn = (double *)malloc(sizeof(double) * nn * d);
  f->bcg = (signed char *)malloc((size_t)nn * d);
  f->u = (double *)calloc((size_t)nn * d, sizeof(double));
  f->vbc = (double *)calloc((size_t)nn * d, sizeof(double));
  return (f->x && f->v && f->B && f->F && f->m && f->vn && f->bcg && f->u && f->vbc) ? OR_OK : OR_E_NOMEM;
}
static void fwd_free(fwd_point *f) {
  free(f->x);
  free(f->v);
  free(f->B);
  free(f->F);
  free(f->m);
  free(f->vn);
  free(f->bcg);
  free(f->u);
  free(f->vbc);
}
static void fwd_save_particles(fwd_point *f, const or_domain *D) {
  const int d = D->dim;
  memcpy(f->x, D->x, sizeof(double) * D->np * d);
  memcpy(f->v, D->v, sizeof(double) * D->np * d);
  memcpy(f->B, D->B, sizeof(double) * D->np * d * d);
  memcpy(f->F, D->F, sizeof(double) * D->np * d * d);
}
static void fwd_save_grid(fwd_point *f, const or_domain *D) {
  memcpy(f->m, D->m, sizeof(double) * nnodes(D));
  memcpy(f->vn, D->vn, sizeof(double) * nnodes(D) * D->dim);
  memcpy(f->bcg, D->bcg, (size_t)nnodes(D) * D->dim);
}
static or_domain fwd_view(const or_domain *D, fwd_point *f) {
  or_domain V = view_of(D, f->x, f->v, f->B, f->F, f->m, f->vn, f->u);
  V.bcg = f->bcg;
  V.vbc = f->vbc;
  return V;
}

/* Adjoint of one single-domain frame (P2G, solve, G2P) of D, which holds the
 * start-of-frame state on entry and the end-of-frame state on exit (the
 * frame is recomputed).  abar_in: adjoint of the end state; abar_out
 * (overwritten): adjoint of the start state; mubar, lambar accumulate. */
int or_single_frame_adjoint(or_domain *D, double dt, const or_solve_opts *opt, double adj_cg_rtol,
                            const double *xb, const double *vb, const double *Bb, const double *Fb,
                            double *oxb, double *ovb, double *oBb, double *oFb, double *mubar,
                            double *lambar) {
  if (is_plastic(D)) return OR_E_ARG;
  const int d = D->dim, nn = nnodes(D), np = D->np;
  fwd_point f0;
  int rc = fwd_alloc(&f0, D);
  double *ubar = (double *)calloc((size_t)nn * d, sizeof(double));
  double *mbar = (double *)calloc((size_t)nn, sizeof(double));
  double *vnbar = (double *)calloc((size_t)nn * d, sizeof(double));
  if (rc || !ubar || !mbar || !vnbar) {
    rc = OR_E_NOMEM;
    goto done;
  }
  fwd_save_particles(&f0, D);
  {
    or_solve_stats st;
    if ((rc = or_p2g(D))) goto done;
    fwd_save_grid(&f0, D);
    D->use_schwarz_bc = 0;
    if ((rc = or_solve(D, dt, opt, &st))) goto done;
    memcpy(f0.u, D->u, sizeof(double) * nn * d);
    if ((rc = or_g2p(D, dt))) goto done;
  }
  memset(oxb, 0, sizeof(double) * np * d);
  memset(ovb, 0, sizeof(double) * np * d);
  memset(oBb, 0, sizeof(double) * np * d * d);
  memset(oFb, 0, sizeof(double) * np * d * d);
  {
    or_domain V = fwd_view(D, &f0);
    V.use_schwarz_bc = 0;
    if ((rc = g2p_adjoint(&V, dt, xb, vb, Bb, Fb, ubar, oxb, oFb))) goto done;
    if ((rc = solve_adjoint(&V, dt, opt->gravity, ubar, adj_cg_rtol, 100000, mbar, vnbar, oxb, oFb, mubar,
                            lambar, NULL)))
      goto done;
    if ((rc = p2g_adjoint(&V, mbar, vnbar, oxb, ovb, oBb))) goto done;
  }
done:
  fwd_free(&f0);
  free(ubar);
  free(mbar);
  free(vnbar);
  return rc;
}

/* Adjoint of one Schwarz frame (Alg. 1) of the pair (B, S), which hold the
 * start-of-frame states on entry and the end-of-frame states on exit.  The
 * frame is recomputed with exactly `iters` Schwarz iterations (the count of
 * the forward run), every intermediate stored, then swept in reverse:
 * coarse G2P; for k = iters-1 .. 0: the projection that fed coarse solve
 * k+1 (through the fine grid after the last sub-step), the M fine sub-steps
 * (P2G, G2P, solve with its Schwarz data, T_m) from last to first, the
 * restore of the stored fine state, both interpolations, v_B = u_B / dT and
 * coarse solve k with its projected data; finally the projection of Step 0
 * and the two Step-0 P2Gs.  Inputs xb*, vb*, Bb*, Fb*: adjoint of the
 * end-of-frame particle states; outputs o* (overwritten): adjoint of the
 * start-of-frame states; mubar*, lambar* accumulate per material.  With
 * `implicit` set the loop over iterations becomes the fixed-point adjoint of
 * or_schwarz_frame_adjoint_implicit (every pass on the last iteration's
 * intermediates, no Step-0 projection). */
static int schwarz_adjoint(or_domain *B, or_domain *S, double dT, const or_schwarz_opts *o, int iters,
                           double adj_cg_rtol, int implicit, double fp_tol, int fp_max, int *fp_used,
                           const double *xbB, const double *vbB, const double *BbB, const double *FbB,
                           const double *xbS, const double *vbS, const double *BbS, const double *FbS,
                           double *oxB, double *ovB, double *oBB, double *oFB, double *oxS, double *ovS,
                           double *oBS, double *oFS, double *mubarB, double *lambarB, double *mubarS,
                           double *lambarS) {
  const int d = B->dim, nnB = nnodes(B), nnS = nnodes(S), npB = B->np, npS = S->np, M = o->M;
  const double dt = dT / (double)M;
  const int K = iters;
  if (K < 1 || M < 1) return OR_E_ARG;
  if (implicit && fp_max < 1) return OR_E_ARG;
  int rc = OR_OK;
  fwd_point fB = {0};
  fwd_point *fS = (fwd_point *)calloc((size_t)K * (M + 1), sizeof(fwd_point));
  double *uB = (double *)calloc((size_t)K * nnB * d, sizeof(double));
  double *piB = (double *)calloc((size_t)K * nnB * d, sizeof(double));
  double *vBk = (double *)malloc(sizeof(double) * nnB * d);
  double *vGSn = (double *)malloc(sizeof(double) * nnS * d);
  double *vGSn1 = (double *)malloc(sizeof(double) * nnS * d);
  double *sx = NULL, *sv = NULL, *sB = NULL, *sF = NULL;
  adj_state aB = {0}, aS0 = {0}, aS = {0}, aP = {0};
  double *ubarB = (double *)calloc((size_t)nnB * d, sizeof(double));
  double *ubarBk = (double *)calloc((size_t)nnB * d, sizeof(double));
  double *mbarB = (double *)calloc((size_t)nnB, sizeof(double));
  double *vnbarB = (double *)calloc((size_t)nnB * d, sizeof(double));
  double *vBkbar = (double *)calloc((size_t)nnB * d, sizeof(double));
  double *pibar = (double *)calloc((size_t)nnB * d, sizeof(double));
  double *pibar_next = (double *)calloc((size_t)nnB * d, sizeof(double));
  double *ubarS = (double *)calloc((size_t)nnS * d, sizeof(double));
  double *mbarS = (double *)calloc((size_t)nnS, sizeof(double));
  double *vnbarS = (double *)calloc((size_t)nnS * d, sizeof(double));
  double *vbcbar = (double *)calloc((size_t)nnS * d, sizeof(double));
  double *gSn = (double *)calloc((size_t)nnS * d, sizeof(double));
  double *gSn1 = (double *)calloc((size_t)nnS * d, sizeof(double));
  if (!fS || !uB || !piB || !vBk || !vGSn || !vGSn1 || !ubarB || !ubarBk || !mbarB || !vnbarB || !vBkbar ||
      !pibar || !pibar_next || !ubarS || !mbarS || !vnbarS || !vbcbar || !gSn || !gSn1) {
    rc = OR_E_NOMEM;
    goto done;
  }
  if ((rc = fwd_alloc(&fB, B))) goto done;
  for (int k = 0; k < K * (M + 1); ++k)
    if ((rc = fwd_alloc(&fS[k], S))) goto done;
  if ((rc = adj_alloc(&aB, npB, d)) || (rc = adj_alloc(&aS0, npS, d)) || (rc = adj_alloc(&aS, npS, d)) ||
      (rc = adj_alloc(&aP, npS, d)))
    goto done;
  sx = (double *)malloc(sizeof(double) * (size_t)(npS > 0 ? npS : 1) * d);
  sv = (double *)malloc(sizeof(double) * (size_t)(npS > 0 ? npS : 1) * d);
  sB = (double *)malloc(sizeof(double) * (size_t)(npS > 0 ? npS : 1) * d * d);
  sF = (double *)malloc(sizeof(double) * (size_t)(npS > 0 ? npS : 1) * d * d);
  if (!sx || !sv || !sB || !sF) {
    rc = OR_E_NOMEM;
    goto done;
  }

  /* ---- forward recompute with storage ---- */
  {
    int n_amb;
    or_solve_stats ss;
    fwd_save_particles(&fB, B);
    memcpy(sx, S->x, sizeof(double) * npS * d);
    memcpy(sv, S->v, sizeof(double) * npS * d);
    memcpy(sB, S->B, sizeof(double) * npS * d * d);
    memcpy(sF, S->F, sizeof(double) * npS * d * d);
    if ((rc = or_p2g(B)) || (rc = or_p2g(S))) goto done;
    fwd_save_grid(&fB, B);
    if ((rc = or_interface(B, S, &n_amb))) goto done;
    if ((rc = or_project(S, B, o->eps_tol, S->vn, &piB[0]))) goto done;
    for (int k = 0; k < K; ++k) {
      memcpy(B->vbc, &piB[(size_t)k * nnB * d], sizeof(double) * nnB * d);
      B->use_schwarz_bc = 1;
      if ((rc = or_solve(B, dT, &o->coarse, &ss))) goto done;
      memcpy(&uB[(size_t)k * nnB * d], B->u, sizeof(double) * nnB * d);
      for (int i = 0; i < nnB; ++i)
        for (int a = 0; a < d; ++a) vBk[i * d + a] = (B->m[i] > 0.0) ? B->u[i * d + a] / dT : 0.0;
      memcpy(S->x, sx, sizeof(double) * npS * d);
      memcpy(S->v, sv, sizeof(double) * npS * d);
      memcpy(S->B, sB, sizeof(double) * npS * d * d);
      memcpy(S->F, sF, sizeof(double) * npS * d * d);
      if ((rc = or_p2g(S))) goto done;
      if ((rc = or_interp(B, fB.vn, S, vGSn))) goto done;
      if ((rc = or_interp(B, vBk, S, vGSn1))) goto done;
      for (int m = 1; m <= M; ++m) {
        fwd_point *f = &fS[k * (M + 1) + (m - 1)];
        fwd_save_particles(f, S);
        fwd_save_grid(f, S);
        or_temporal(nnS * d, m, M, vGSn, vGSn1, S->vbc);
        memcpy(f->vbc, S->vbc, sizeof(double) * nnS * d);
        S->use_schwarz_bc = 1;
        if ((rc = or_solve(S, dt, &o->fine, &ss))) goto done;
        memcpy(f->u, S->u, sizeof(double) * nnS * d);
        if ((rc = or_g2p(S, dt))) goto done;
        if ((rc = or_p2g(S))) goto done;
      }
      fwd_point *fl = &fS[k * (M + 1) + M];
      fwd_save_particles(fl, S);
      fwd_save_grid(fl, S);
      if (k + 1 < K)
        if ((rc = or_project(S, B, o->eps_tol, S->vn, &piB[(size_t)(k + 1) * nnB * d]))) goto done;
    }
    memcpy(B->u, &uB[(size_t)(K - 1) * nnB * d], sizeof(double) * nnB * d);
    if ((rc = or_g2p(B, dT))) goto done;
  }

  /* ---- reverse sweep ---- */
  {
    const double *grB = o->coarse.gravity, *grS = o->fine.gravity;
    or_domain VB = view_of(B, fB.x, fB.v, fB.B, fB.F, fB.m, fB.vn, &uB[(size_t)(K - 1) * nnB * d]);
    VB.bcg = fB.bcg;
    VB.use_schwarz_bc = 1;
    /* coarse G2P */
    if ((rc = g2p_adjoint(&VB, dT, xbB, vbB, BbB, FbB, ubarB, aB.x, aB.F))) goto done;
    double w_norm = 0.0;
    for (int j = 0;; ++j) {
      /* unrolled: iteration k = K-1-j; implicit: always the last iterate */
      const int k = implicit ? K - 1 : K - 1 - j;
      if (k < 0) break;
      memset(ubarBk, 0, sizeof(double) * nnB * d);
      if (j == 0) memcpy(ubarBk, ubarB, sizeof(double) * nnB * d);
      /* adjoint of the fine state after the last sub-step of iteration k */
      if (j == 0) {
        memcpy(aS.x, xbS, sizeof(double) * npS * d);
        memcpy(aS.v, vbS, sizeof(double) * npS * d);
        memcpy(aS.B, BbS, sizeof(double) * npS * d * d);
        memcpy(aS.F, FbS, sizeof(double) * npS * d * d);
      } else {
        adj_zero(&aS, npS, d);
        /* the projection of this grid fed coarse solve k+1 */
        or_domain VL = fwd_view(S, &fS[k * (M + 1) + M]);
        memset(mbarS, 0, sizeof(double) * nnS);
        memset(vnbarS, 0, sizeof(double) * nnS * d);
        if ((rc = project_adjoint(&VL, B, o->eps_tol, pibar_next, mbarS, vnbarS))) goto done;
        if ((rc = p2g_adjoint(&VL, mbarS, vnbarS, aS.x, aS.v, aS.B))) goto done;
      }
      memset(gSn, 0, sizeof(double) * nnS * d);
      memset(gSn1, 0, sizeof(double) * nnS * d);
      for (int m = M; m >= 1; --m) {
        fwd_point *f = &fS[k * (M + 1) + (m - 1)];
        or_domain V = fwd_view(S, f);
        V.use_schwarz_bc = 1;
        adj_zero(&aP, npS, d);
        memset(ubarS, 0, sizeof(double) * nnS * d);
        if ((rc = g2p_adjoint(&V, dt, aS.x, aS.v, aS.B, aS.F, ubarS, aP.x, aP.F))) goto done;
        memset(mbarS, 0, sizeof(double) * nnS);
        memset(vnbarS, 0, sizeof(double) * nnS * d);
        memset(vbcbar, 0, sizeof(double) * nnS * d);
        if ((rc = solve_adjoint(&V, dt, grS, ubarS, adj_cg_rtol, 100000, mbarS, vnbarS, aP.x, aP.F, mubarS,
                                lambarS, vbcbar)))
          goto done;
        const double am = (double)m / (double)M;
        for (int q = 0; q < nnS * d; ++q) {
          gSn[q] += (1.0 - am) * vbcbar[q];
          gSn1[q] += am * vbcbar[q];
        }
        if ((rc = p2g_adjoint(&V, mbarS, vnbarS, aP.x, aP.v, aP.B))) goto done;
        adj_state t = aS;
        aS = aP;
        aP = t;
      }
      /* restore: the stored fine state */
      for (int q = 0; q < npS * d; ++q) {
        aS0.x[q] += aS.x[q];
        aS0.v[q] += aS.v[q];
      }
      for (int q = 0; q < npS * d * d; ++q) {
        aS0.B[q] += aS.B[q];
        aS0.F[q] += aS.F[q];
      }
      /* interpolations: I(v_B^(k+1)) and I(v_B^n) */
      memset(vBkbar, 0, sizeof(double) * nnB * d);
      if ((rc = interp_adjoint(&VB, S, gSn1, vBkbar))) goto done;
      if ((rc = interp_adjoint(&VB, S, gSn, vnbarB))) goto done;
      for (int i = 0; i < nnB; ++i)
        if (fB.m[i] > 0.0)
          for (int a = 0; a < d; ++a) ubarBk[i * d + a] += vBkbar[i * d + a] / dT;
      /* coarse solve k */
      VB.u = &uB[(size_t)k * nnB * d];
      VB.vbc = &piB[(size_t)k * nnB * d];
      memset(pibar, 0, sizeof(double) * nnB * d);
      if ((rc = solve_adjoint(&VB, dT, grB, ubarBk, adj_cg_rtol, 100000, mbarB, vnbarB, aB.x, aB.F, mubarB,
                              lambarB, pibar)))
        goto done;
      memcpy(pibar_next, pibar, sizeof(double) * nnB * d);
      if (implicit) {
        /* pibar is now (Phi_z^T)^j w, w = pibar of j = 0 */
        double nrm = 0.0;
        for (int q = 0; q < nnB * d; ++q) nrm += pibar[q] * pibar[q];
        nrm = sqrt(nrm);
        if (j == 0) w_norm = nrm;
        *fp_used = j;
        if (fp_tol > 0.0 && nrm <= fp_tol * w_norm) break;
        if (j == fp_max) {
          if (fp_tol > 0.0) rc = OR_E_NOT_CONVERGED;
          break;
        }
      }
    }
    if (rc) goto done;
    /* Step 0: projection of the fine start grid (the first iterate's
     * Dirichlet data; the fixed point does not depend on it), then both
     * P2Gs */
    if (!implicit) {
      or_domain V0 = fwd_view(S, &fS[0]);
      memset(mbarS, 0, sizeof(double) * nnS);
      memset(vnbarS, 0, sizeof(double) * nnS * d);
      if ((rc = project_adjoint(&V0, B, o->eps_tol, pibar_next, mbarS, vnbarS))) goto done;
      if ((rc = p2g_adjoint(&V0, mbarS, vnbarS, aS0.x, aS0.v, aS0.B))) goto done;
    }
    if ((rc = p2g_adjoint(&VB, mbarB, vnbarB, aB.x, aB.v, aB.B))) goto done;
    memcpy(oxB, aB.x, sizeof(double) * npB * d);
    memcpy(ovB, aB.v, sizeof(double) * npB * d);
    memcpy(oBB, aB.B, sizeof(double) * npB * d * d);
    memcpy(oFB, aB.F, sizeof(double) * npB * d * d);
    memcpy(oxS, aS0.x, sizeof(double) * npS * d);
    memcpy(ovS, aS0.v, sizeof(double) * npS * d);
    memcpy(oBS, aS0.B, sizeof(double) * npS * d * d);
    memcpy(oFS, aS0.F, sizeof(double) * npS * d * d);
  }
done:
  if (fS) {
    for (int k = 0; k < K * (M + 1); ++k) fwd_free(&fS[k]);
    free(fS);
  }
  fwd_free(&fB);
  free(uB);
  free(piB);
  free(vBk);
  free(vGSn);
  free(vGSn1);
  free(sx);
  free(sv);
  free(sB);
  free(sF);
  adj_free(&aB);
  adj_free(&aS0);
  adj_free(&aS);
  adj_free(&aP);
  free(ubarB);
  free(ubarBk);
  free(mbarB);
  free(vnbarB);
  free(vBkbar);
  free(pibar);
  free(pibar_next);
  free(ubarS);
  free(mbarS);
  free(vnbarS);
  free(vbcbar);
  free(gSn);
  free(gSn1);
  return rc;
}

int or_schwarz_frame_adjoint(or_domain *B, or_domain *S, double dT, const or_schwarz_opts *o, int iters,
                             double adj_cg_rtol, const double *xbB, const double *vbB, const double *BbB,
                             const double *FbB, const double *xbS, const double *vbS, const double *BbS,
                             const double *FbS, double *oxB, double *ovB, double *oBB, double *oFB,
                             double *oxS, double *ovS, double *oBS, double *oFS, double *mubarB,
                             double *lambarB, double *mubarS, double *lambarS) {
  if (is_plastic(B) || is_plastic(S)) return OR_E_ARG;
  int unused = 0;
  return schwarz_adjoint(B, S, dT, o, iters, adj_cg_rtol, 0, 0.0, 0, &unused, xbB, vbB, BbB, FbB, xbS, vbS,
                         BbS, FbS, oxB, ovB, oBB, oFB, oxS, ovS, oBS, oFS, mubarB, lambarB, mubarS, lambarS);
}

/* Implicit (fixed-point) adjoint of the Schwarz iteration.  Alg. 1 iterates
 * z -> Phi(z; theta), z the projected Dirichlet data of the coarse solve and
 * theta the start-of-frame states and materials; the outputs are psi(z; theta)
 * (the coarse solve with data z, its G2P, and the fine sub-steps driven by
 * it).  At the fixed point z* = Phi(z*), dL/dtheta = psi_theta^T obar +
 * Phi_theta^T mu with (I - Phi_z^T) mu = psi_z^T obar, which the Neumann
 * series mu = sum_j (Phi_z^T)^j w solves at the contraction rate of the
 * forward iteration (Sec. 2.3: for a coercive problem the Schwarz iteration
 * contracts geometrically, Phi_z^T with it).  Every term is linearised at the last forward
 * iterate, so only that iteration's intermediates are needed, and the first
 * iterate's data (the Step-0 projection) drops out.  The frame is recomputed
 * with `iters` Schwarz iterations.  fp_tol > 0: stop once the 2-norm of
 * (Phi_z^T)^j w falls to fp_tol times that of w, at most fp_max applications
 * of Phi_z^T (else OR_E_NOT_CONVERGED); fp_tol <= 0: exactly fp_max.  fp_used
 * receives the number of applications. */
int or_schwarz_frame_adjoint_implicit(or_domain *B, or_domain *S, double dT, const or_schwarz_opts *o,
                                      int iters, double adj_cg_rtol, double fp_tol, int fp_max, int *fp_used,
                                      const double *xbB, const double *vbB, const double *BbB,
                                      const double *FbB, const double *xbS, const double *vbS,
                                      const double *BbS, const double *FbS, double *oxB, double *ovB,
                                      double *oBB, double *oFB, double *oxS, double *ovS, double *oBS,
                                      double *oFS, double *mubarB, double *lambarB, double *mubarS,
                                      double *lambarS) {
  if (is_plastic(B) || is_plastic(S)) return OR_E_ARG;
  return schwarz_adjoint(B, S, dT, o, iters, adj_cg_rtol, 1, fp_tol, fp_max, fp_used, xbB, vbB, BbB, FbB, xbS,
                         vbS, BbS, FbS, oxB, ovB, oBB, oFB, oxS, ovS, oBS, oFS, mubarB, lambarB, mubarS,
                         lambarS);
}
