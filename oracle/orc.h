/*
 * Plain CPU FP64 oracle for classical-AMG-preconditioned CG.
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the GPU library
 * against an independent, slow, obviously-correct implementation written
 * from the paper (Isotton, Frigo, Spiezia, Janna, "Chronos: a general
 * purpose classical AMG solver for High Performance Computing").  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source with the GPU library.
 *
 * Single-threaded, compiled with -O2 -ffp-contract=off so every multiply and
 * add is rounded separately in the order written.
 *
 * Status codes (same meaning as the GPU library's, defined independently):
 *   0 OK, 1 MAXIT (outputs valid), -1 bad argument, -2 malformed CSR,
 *   -3 not SPD (non-positive diagonal or Cholesky pivot), -4 CG breakdown,
 *   -5 coarsest level too large, -6 out of memory.
 */
#ifndef CAMG_ORACLE_H
#define CAMG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_MAXIT = 1, ORC_E_ARG = -1, ORC_E_CSR = -2, ORC_E_NOT_SPD = -3,
       ORC_E_BREAKDOWN = -4, ORC_E_COARSE = -5, ORC_E_NOMEM = -6 };

/* C/F markers */
enum { ORC_F = -1, ORC_U = 0, ORC_C = 1 };

typedef struct {
    int32_t nrows, ncols;
    int32_t *rp;     /* nrows+1 */
    int32_t *ci;     /* nnz, ascending per row */
    double  *val;    /* nnz */
} orc_csr;

typedef struct {
    double   theta;       /* strength threshold (0.25) */
    uint64_t seed;        /* PMIS random seed */
    int32_t  nu_pre, nu_post;
    double   omega;       /* <= 0: (4/3)/Gershgorin bound per level */
    int32_t  max_levels;
    int32_t  max_coarse;
    int32_t  max_iter;
    int32_t  smoother;    /* ORC_SMOOTH_JACOBI (M = D), ORC_SMOOTH_FSAI (M^{-1} = G^T G, static G),
                             ORC_SMOOTH_FSAI_JACOBI (FSAI per level where the rows are short enough) or
                             ORC_SMOOTH_AFSAI (M^{-1} = G^T G, adaptive G) */
    int32_t  interp;      /* ORC_INTERP_* */
    int32_t  bamg_lmin, bamg_lmax;  /* BAMG: interpolation distances tried (1, 2) */
    double   bamg_eps, bamg_mu;     /* BAMG: accept when relative residual <= eps and ||w|| <= mu */
    int32_t  psmooth;     /* 1: one Jacobi step on P (P - omega D^{-1} A P) */
    double   pfilter;     /* < 1: filter P, keeping this fraction of each row's absolute sum */
    int32_t  srqm_iters;  /* BAMG: SRQM steps refining the level-0 test space (0: none) */
    int32_t  afsai_steps; /* ORC_SMOOTH_AFSAI: growth steps per row (steps * step + 1 <= ORC_AFSAI_MAXM) */
    int32_t  afsai_step;  /*   entries added per step */
    double   afsai_eps;   /*   stop a row when psi_i falls by no more than this fraction in a step */
} orc_params;
enum { ORC_SMOOTH_JACOBI = 0, ORC_SMOOTH_FSAI = 1, ORC_SMOOTH_FSAI_JACOBI = 2, ORC_SMOOTH_AFSAI = 3 };
#define ORC_AFSAI_MAXM 32        /* entries of a row of the adaptive factor */
#define ORC_FSAI_POWER_STEPS 15  /* power steps of the FSAI relaxation weight's estimate of rho(G A G^T) */
#define ORC_AFSAI_MAXCAND 2048   /* ORC_SMOOTH_AFSAI: a level where a row's candidate set grows larger uses Jacobi */
#define ORC_FSAI_MAXROW 192  /* ORC_SMOOTH_FSAI_JACOBI: FSAI on levels whose rows have at most this many
                                entries on or below the diagonal, Jacobi on the others */
enum { ORC_INTERP_DIRECT = 0, ORC_INTERP_CLASSICAL = 1, ORC_INTERP_EXTI = 2, ORC_INTERP_HYBRID = 3,
       ORC_INTERP_BAMG = 4 };
#define ORC_MAXNT 8        /* test vectors */
#define ORC_MAXCAND 4096   /* BAMG candidates of one row */

void orc_params_default(orc_params *p);

/* ---- single steps (each on caller buffers unless it returns a CSR) ---- */
int  orc_validate(int32_t n, const int32_t *rp, const int32_t *ci, const double *v);
void orc_strength(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                  double theta, uint8_t *strong, int32_t *st_count);
uint64_t orc_splitmix64(uint64_t seed, uint64_t counter);
uint64_t orc_pmis_rand(uint64_t seed, int32_t level, int32_t i);
int  orc_pmis(int32_t n, const int32_t *rp, const int32_t *ci, const uint8_t *strong,
              const int32_t *st_count, uint64_t seed, int32_t level, int8_t *cf, int32_t *rounds);
int  orc_interp_direct(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                       const uint8_t *strong, const int8_t *cf, orc_csr *P);
/* classical (a_ij restored), extended+i or hybrid interpolation for a given C/F split */
int  orc_interp(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                const uint8_t *strong, const int8_t *cf, int32_t variant, orc_csr *P);
/* BAMG: orthonormal basis of a test space V (n x nt, row-major, in place) */
int  orc_orthonormalize(int32_t n, int32_t nt, double *V);
/* BAMG prolongation for test space V (n x nt) and a given C/F split */
int  orc_bamg(int32_t n, const int32_t *rp, const int32_t *ci, const uint8_t *strong, const int8_t *cf, int32_t nt,
              const double *V, int32_t lmin, int32_t lmax, double eps, double mu, orc_csr *P);
/* prolongation smoothing P - omega D^{-1} A P, and filtering with compensation on W (nc x nt) */
int  orc_psmooth(const orc_csr *A, const double *dinv, double omega, const orc_csr *P, orc_csr *Ps);
int  orc_pfilter(const orc_csr *P, double rho, int32_t nt, const double *W, orc_csr *Pf);
/* eigen-decomposition of a symmetric m x m matrix (m <= 2 ORC_MAXNT; C overwritten) by cyclic Jacobi */
int  orc_symeig(int32_t m, double *C, double *lam, double *Q);
/* SRQM refinement of an orthonormal test space V (n x nt, in place) with M^{-1} = D^{-1}, or G^T G if G */
int  orc_srqm(const orc_csr *A, const double *dinv, const orc_csr *G, const orc_csr *GT, int32_t nt, double *V,
              int32_t iters, int32_t *done);
int  orc_transpose(const orc_csr *X, orc_csr *XT);
int  orc_spgemm(const orc_csr *X, const orc_csr *Y, orc_csr *Z);
int  orc_cholesky(int32_t n, double *a);      /* in: dense SPD row-major; out: L in the lower triangle */
void orc_chol_solve(int32_t n, const double *L, const double *y, double *z);
double orc_gershgorin_omega(int32_t n, const int32_t *rp, const int32_t *ci, const double *v);
/* static FSAI factor G (lower triangular, pattern of the lower triangle of A) */
int  orc_fsai(const orc_csr *A, orc_csr *G);
/* adaptive FSAI factor (pattern grown greedily by the Kaporin gradient); *maxcand: largest candidate set */
int  orc_afsai(const orc_csr *A, int32_t steps, int32_t step, double eps, orc_csr *G, int32_t *maxcand);
/* the same for the rows sel[0..nsel) only: row t in cols / vals[t * (steps * step + 1) ...], count in cnt[t] */
int  orc_afsai_rows(const orc_csr *A, int32_t steps, int32_t step, double eps, int32_t nsel, const int32_t *sel,
                    int32_t *cols, double *vals, int32_t *cnt, int32_t *maxcand);
/* omega = (4/3) / max_i sum_j |(G A G^T)_ij| */
int  orc_fsai_omega(const orc_csr *A, const orc_csr *G, uint64_t seed, int32_t level, double *omega);
void orc_csr_free(orc_csr *m);
void orc_free(void *p);

/* ---- hierarchy and solver ---- */
typedef struct orc_hier orc_hier;
int  orc_setup(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
               const orc_params *prm, orc_hier **out);
/* the same with a test space V (n x nt, row-major; needed by ORC_INTERP_BAMG) */
int  orc_setup_tv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nt, const double *V,
                  const orc_params *prm, orc_hier **out);
int  orc_num_levels(const orc_hier *h);
/* sizes of level l: n, nnz(A), nnz(P) (0 on the coarsest), n of level l+1 (0 on the coarsest) */
int  orc_level_sizes(const orc_hier *h, int32_t l, int32_t *n, int32_t *nnzA, int32_t *nnzP, int32_t *nc);
enum { ORC_X_A = 0, ORC_X_P = 1, ORC_X_R = 2, ORC_X_CF = 3, ORC_X_STRONG = 4, ORC_X_DINV = 5,
       ORC_X_OMEGA = 6, ORC_X_CHOL = 7, ORC_X_STCNT = 8, ORC_X_ROUNDS = 9, ORC_X_G = 10 };
int  orc_export(const orc_hier *h, int32_t l, int32_t what, void *a, void *b, void *c);
/* z = M y : one V-cycle */
void orc_vcycle(const orc_hier *h, const double *y, double *z);
/* PCG from x0 = 0; precond: 1 = AMG V-cycle, 0 = identity */
int  orc_solve(const orc_hier *h, const double *b, double rtol, int32_t max_iter, int32_t precond,
               double *x, int32_t *iters, double *hist, int32_t hist_cap, double *true_relres);
void orc_destroy(orc_hier *h);

#ifdef __cplusplus
}
#endif
#endif
