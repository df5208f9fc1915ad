// Solve-phase kernels: the V-cycle of Alg. "AMG application in a V-cycle"
// with Jacobi smoothing (eq. smoother, M = D) and the PCG recurrence.
//
// All of them are CSR row kernels: a group of `LPR` lanes (1..64) walks one
// row, with LPR chosen per matrix from its mean row length; each block owns
// one contiguous range of rows and blocks are renumbered so that one XCD
// works on one contiguous slab of the matrix (its L2 then holds the gathered
// vector entries its rows share).  The CG dot products are fused into the
// kernels that produce their operands: each block writes one partial sum and
// the last block to finish adds the partials in index order, so every
// reduction is deterministic.  Scalars of the recurrence (alpha, beta, rho,
// ...) stay in device memory; once the residual test passes the kernels see
// `done` and return at once.
#include "devutil.hpp"
#include "internal.hpp"

namespace camg {

namespace {

template <int LPR>
struct Rows {
    static constexpr int RPB = kBlock / LPR;  // rows per pass of one block
    int r0, r1;
    __device__ Rows(int n, int rows_per_block) {
        const int b = xcd_block();
        r0 = min(n, b * rows_per_block);
        r1 = min(n, r0 + rows_per_block);
    }
};

__device__ __forceinline__ int sub_lane(int lpr) { return threadIdx.x & (lpr - 1); }

// ------------------------------------------------------------------ V-cycle
// pre-smoothing from s = 0 fused with the residual:
//   s_i = wd_i y_i,  r_i = y_i - sum_j a_ij (wd_j y_j)
template <class T, class TY, int LPR>
__global__ void __launch_bounds__(kBlock) k_vc_pre(int n, int rpb, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const T *__restrict__ av,
                                                   const T *__restrict__ wd, const TY *__restrict__ y,
                                                   T *__restrict__ s, T *__restrict__ r, const PcgState *st) {
    if (st && st->done) return;
    Rows<LPR> R(n, rpb);
    const int sl = sub_lane(LPR), g = threadIdx.x / LPR;
    for (int base = R.r0; base < R.r1; base += Rows<LPR>::RPB) {
        const int i = base + g;
        T acc = 0;
        if (i < R.r1) {
            const int e1 = rp[i + 1];
            for (int e = rp[i] + sl; e < e1; e += LPR) {
                const int j = ci[e];
                acc += av[e] * (wd[j] * (T)y[j]);
            }
        }
        acc = group_sum<LPR>(acc);
        if (i < R.r1 && sl == 0) {
            const T yi = (T)y[i];
            s[i] = wd[i] * yi;
            r[i] = yi - acc;
        }
    }
}

// one Jacobi step z = s + wd (y - A s); with DOT the block also adds y_i z_i
// (level 0: y is the PCG residual) and the last block forms rho and beta.
template <class T, class TY, class TZ, int LPR, bool DOT>
__global__ void __launch_bounds__(kBlock) k_vc_post(int n, int rpb, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci, const T *__restrict__ av,
                                                    const T *__restrict__ wd, const TY *__restrict__ y,
                                                    const T *__restrict__ s, TZ *__restrict__ z, double *partials,
                                                    unsigned *counter, PcgState *st) {
    if (st && st->done) return;
    Rows<LPR> R(n, rpb);
    const int sl = sub_lane(LPR), g = threadIdx.x / LPR;
    double dot = 0.0;
    for (int base = R.r0; base < R.r1; base += Rows<LPR>::RPB) {
        const int i = base + g;
        T acc = 0;
        if (i < R.r1) {
            const int e1 = rp[i + 1];
            for (int e = rp[i] + sl; e < e1; e += LPR) acc += av[e] * s[ci[e]];
        }
        acc = group_sum<LPR>(acc);
        if (i < R.r1 && sl == 0) {
            const T yi = (T)y[i];
            const T zi = s[i] + wd[i] * (yi - acc);
            z[i] = (TZ)zi;
            if (DOT) dot += (double)y[i] * (double)(TZ)zi;
        }
    }
    if (DOT) {
        const double b = block_sum<kBlock>(dot);
        if (threadIdx.x == 0) partials[blockIdx.x] = b;
        if (last_block(counter)) {
            const double rho = sum_partials<kBlock>(partials, gridDim.x);
            if (threadIdx.x == 0) {
                st->rho = rho;
                st->beta = st->iter == 0 ? 0.0 : rho / st->rho_old;
                *counter = 0;
            }
        }
    }
}

// r = y - A s (after extra pre-smoothing steps)
template <class T, class TY, int LPR>
__global__ void __launch_bounds__(kBlock) k_vc_resid(int n, int rpb, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, const T *__restrict__ av,
                                                     const TY *__restrict__ y, const T *__restrict__ s,
                                                     T *__restrict__ r, const PcgState *st) {
    if (st && st->done) return;
    Rows<LPR> R(n, rpb);
    const int sl = sub_lane(LPR), g = threadIdx.x / LPR;
    for (int base = R.r0; base < R.r1; base += Rows<LPR>::RPB) {
        const int i = base + g;
        T acc = 0;
        if (i < R.r1) {
            const int e1 = rp[i + 1];
            for (int e = rp[i] + sl; e < e1; e += LPR) acc += av[e] * s[ci[e]];
        }
        acc = group_sum<LPR>(acc);
        if (i < R.r1 && sl == 0) r[i] = (T)y[i] - acc;
    }
}

// out = M x (ADD: out += M x)
template <class T, int LPR, bool ADD>
__global__ void __launch_bounds__(kBlock) k_spmv(int n, int rpb, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const T *__restrict__ mv,
                                                 const T *__restrict__ x, T *__restrict__ out, const PcgState *st) {
    if (st && st->done) return;
    Rows<LPR> R(n, rpb);
    const int sl = sub_lane(LPR), g = threadIdx.x / LPR;
    for (int base = R.r0; base < R.r1; base += Rows<LPR>::RPB) {
        const int i = base + g;
        T acc = 0;
        if (i < R.r1) {
            const int e1 = rp[i + 1];
            for (int e = rp[i] + sl; e < e1; e += LPR) acc += mv[e] * x[ci[e]];
        }
        acc = group_sum<LPR>(acc);
        if (i < R.r1 && sl == 0) out[i] = ADD ? out[i] + acc : acc;
    }
}

// last level: z = Ainv y, one wavefront per row, FP64 arithmetic
template <class T>
__global__ void __launch_bounds__(kBlock) k_coarse(int n, const double *__restrict__ cinv, const T *__restrict__ y,
                                                   T *__restrict__ z, const PcgState *st) {
    if (st && st->done) return;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc += cinv[(int64_t)i * n + j] * (double)y[j];
    acc = wave_sum(acc);
    if (lane == 0) z[i] = (T)acc;
}

// rho = y . z for a one-level hierarchy (no smoothing kernel to fuse into)
__global__ void __launch_bounds__(kBlock) k_dot_rho(int n, const double *__restrict__ y, const double *__restrict__ z,
                                                    double *partials, unsigned *counter, PcgState *st) {
    if (st->done) return;
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) acc += y[i] * z[i];
    const double b = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
    if (last_block(counter)) {
        const double rho = sum_partials<kBlock>(partials, gridDim.x);
        if (threadIdx.x == 0) {
            st->rho = rho;
            st->beta = st->iter == 0 ? 0.0 : rho / st->rho_old;
            *counter = 0;
        }
    }
}

// ------------------------------------------------------------------ PCG
__global__ void __launch_bounds__(kBlock) k_pcg_init(int n, const double *__restrict__ b, double *__restrict__ x,
                                                     double *__restrict__ r, double *__restrict__ p0, double rtol,
                                                     double *partials, unsigned *counter, PcgState *st,
                                                     double *hist) {
    double acc = 0.0;
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        p0[i] = 0.0;
        acc += bi * bi;
    }
    const double bs = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    if (last_block(counter)) {
        const double b2 = sum_partials<kBlock>(partials, gridDim.x);
        if (threadIdx.x == 0) {
            const double bn = sqrt(b2);
            st->bnorm = bn;
            st->rnorm = bn;
            st->tol = rtol > 0.0 ? rtol * bn : -1.0;
            st->rho = st->rho_old = st->sigma = st->alpha = st->beta = 0.0;
            st->iter = 0;
            st->status = 0;
            st->done = (bn == 0.0 || bn < st->tol) ? 1 : 0;
            hist[0] = bn;
            *counter = 0;
        }
    }
}

// p_new = z + beta p_old (p_new = z on the first iteration), q = A p_new,
// sigma = p_new . q, alpha = rho / sigma; the neighbours' p_new entries are
// formed on the fly from z and p_old (the same rounded expression).
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_pcg_spmv_p(int n, int rpb, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, const double *__restrict__ av,
                                                       const double *__restrict__ z, const double *__restrict__ pold,
                                                       double *__restrict__ pnew, double *__restrict__ q,
                                                       double *partials, unsigned *counter, PcgState *st) {
    if (st->done) return;
    const bool first = st->iter == 0;
    const double beta = st->beta;
    Rows<LPR> R(n, rpb);
    const int sl = sub_lane(LPR), g = threadIdx.x / LPR;
    double dot = 0.0;
    for (int base = R.r0; base < R.r1; base += Rows<LPR>::RPB) {
        const int i = base + g;
        double acc = 0.0;
        if (i < R.r1) {
            const int e1 = rp[i + 1];
            if (first)
                for (int e = rp[i] + sl; e < e1; e += LPR) acc += av[e] * z[ci[e]];
            else
                for (int e = rp[i] + sl; e < e1; e += LPR) {
                    const int j = ci[e];
                    acc += av[e] * (z[j] + beta * pold[j]);
                }
        }
        acc = group_sum<LPR>(acc);
        if (i < R.r1 && sl == 0) {
            const double pi = first ? z[i] : z[i] + beta * pold[i];
            pnew[i] = pi;
            q[i] = acc;
            dot += pi * acc;
        }
    }
    const double bsum = block_sum<kBlock>(dot);
    if (threadIdx.x == 0) partials[blockIdx.x] = bsum;
    if (last_block(counter)) {
        const double sigma = sum_partials<kBlock>(partials, gridDim.x);
        if (threadIdx.x == 0) {
            st->sigma = sigma;
            if (!(sigma > 0.0) || !(st->rho > 0.0)) {
                st->status = (int32_t)CAMG_E_BREAKDOWN;
                st->done = 1;
            } else {
                st->alpha = st->rho / sigma;
            }
            *counter = 0;
        }
    }
}

// x += alpha p, r -= alpha q, ||r||; convergence test on the recursive residual
__global__ void __launch_bounds__(kBlock) k_pcg_update(int n, const double *__restrict__ p,
                                                       const double *__restrict__ q, double *__restrict__ x,
                                                       double *__restrict__ r, double *partials, unsigned *counter,
                                                       PcgState *st, double *hist, int hist_cap, int32_t *hflag) {
    if (st->done) return;
    const double alpha = st->alpha;
    double acc = 0.0;
    const int stride = gridDim.x * kBlock;
    for (int i = xcd_block() * kBlock + threadIdx.x; i < n; i += stride) {
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    const double bs = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    if (last_block(counter)) {
        const double r2 = sum_partials<kBlock>(partials, gridDim.x);
        if (threadIdx.x == 0) {
            const double rn = sqrt(r2);
            const int it = st->iter + 1;
            st->iter = it;
            st->rnorm = rn;
            st->rho_old = st->rho;
            if (it < hist_cap) hist[it] = rn;
            if (st->tol > 0.0 && rn < st->tol) st->done = 1;
            if (hflag) hflag[0] = st->done;
            *counter = 0;
        }
    }
}

// ||b - A x||^2 into *out2
template <int LPR>
__global__ void __launch_bounds__(kBlock) k_true_res(int n, int rpb, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, const double *__restrict__ av,
                                                     const double *__restrict__ b, const double *__restrict__ x,
                                                     double *partials, unsigned *counter, double *out2) {
    Rows<LPR> R(n, rpb);
    const int sl = sub_lane(LPR), g = threadIdx.x / LPR;
    double loc = 0.0;
    for (int base = R.r0; base < R.r1; base += Rows<LPR>::RPB) {
        const int i = base + g;
        double acc = 0.0;
        if (i < R.r1) {
            const int e1 = rp[i + 1];
            for (int e = rp[i] + sl; e < e1; e += LPR) acc += av[e] * x[ci[e]];
        }
        acc = group_sum<LPR>(acc);
        if (i < R.r1 && sl == 0) {
            const double d = b[i] - acc;
            loc += d * d;
        }
    }
    const double bs = block_sum<kBlock>(loc);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    if (last_block(counter)) {
        const double t = sum_partials<kBlock>(partials, gridDim.x);
        if (threadIdx.x == 0) {
            *out2 = t;
            *counter = 0;
        }
    }
}

__global__ void k_fill_zero(int64_t n, double *x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// ------------------------------------------------------------------ dispatch
int rows_per_block(int n, const RowCfg &c, int grid) {
    const int rpp = kBlock / c.lpr;
    const int per = (n + grid - 1) / grid;
    return ((per + rpp - 1) / rpp) * rpp;
}

#define CAMG_LPR_SWITCH(lpr, ...)                      \
    switch (lpr) {                                     \
    case 1: { constexpr int L = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int L = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int L = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int L = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int L = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int L = 32; __VA_ARGS__; } break; \
    default: { constexpr int L = 64; __VA_ARGS__; } break; \
    }

}  // namespace

RowCfg choose_cfg(int n, int64_t nnz) {
    RowCfg c;
    const double mean = n > 0 ? (double)nnz / n : 1.0;
    int l = 1;
    while (l < 64 && l < mean) l <<= 1;
    c.lpr = l;
    return c;
}

int grid_for(int n, const RowCfg &c) {
    const int rpp = kBlock / c.lpr;
    int g = (n + rpp - 1) / rpp;
    g = std::min(g, kMaxGrid);
    g = std::max(8, (g + 7) / 8 * 8);
    return g;
}

template <class T>
static const T *vals(const Csr &A);
template <>
const double *vals<double>(const Csr &A) { return A.v; }
template <>
const float *vals<float>(const Csr &A) { return A.v32; }

template <class T, class TY>
void vc_pre(const Csr &A, const RowCfg &c, const T *wd, const TY *y, T *s, T *r, const PcgState *st,
            hipStream_t str) {
    const int g = grid_for(A.nr, c), rpb = rows_per_block(A.nr, c, g);
    CAMG_LPR_SWITCH(c.lpr, (k_vc_pre<T, TY, L><<<g, kBlock, 0, str>>>(A.nr, rpb, A.rp, A.ci, vals<T>(A), wd, y, s, r, st)));
    HIPC(hipGetLastError());
}

template <class T, class TY, class TZ, bool DOT>
void vc_post(const Csr &A, const RowCfg &c, const T *wd, const TY *y, const T *s, TZ *z, double *partials,
             unsigned *counter, PcgState *st, hipStream_t str) {
    const int g = grid_for(A.nr, c), rpb = rows_per_block(A.nr, c, g);
    CAMG_LPR_SWITCH(c.lpr, (k_vc_post<T, TY, TZ, L, DOT><<<g, kBlock, 0, str>>>(A.nr, rpb, A.rp, A.ci, vals<T>(A), wd,
                                                                                    y, s, z, partials, counter, st)));
    HIPC(hipGetLastError());
}

template <class T, class TY>
void vc_resid(const Csr &A, const RowCfg &c, const TY *y, const T *s, T *r, const PcgState *st, hipStream_t str) {
    const int g = grid_for(A.nr, c), rpb = rows_per_block(A.nr, c, g);
    CAMG_LPR_SWITCH(c.lpr, (k_vc_resid<T, TY, L><<<g, kBlock, 0, str>>>(A.nr, rpb, A.rp, A.ci, vals<T>(A), y, s, r, st)));
    HIPC(hipGetLastError());
}
template <class T>
void vc_restrict(const Csr &R, const RowCfg &c, const T *r, T *yc, const PcgState *st, hipStream_t str) {
    const int g = grid_for(R.nr, c), rpb = rows_per_block(R.nr, c, g);
    CAMG_LPR_SWITCH(c.lpr, (k_spmv<T, L, false><<<g, kBlock, 0, str>>>(R.nr, rpb, R.rp, R.ci, vals<T>(R), r, yc, st)));
    HIPC(hipGetLastError());
}
template <class T>
void vc_prolong(const Csr &P, const RowCfg &c, const T *d, T *s, const PcgState *st, hipStream_t str) {
    const int g = grid_for(P.nr, c), rpb = rows_per_block(P.nr, c, g);
    CAMG_LPR_SWITCH(c.lpr, (k_spmv<T, L, true><<<g, kBlock, 0, str>>>(P.nr, rpb, P.rp, P.ci, vals<T>(P), d, s, st)));
    HIPC(hipGetLastError());
}
template <class T>
void coarse_solve(int n, const double *cinv, const T *y, T *z, const PcgState *st, hipStream_t str) {
    k_coarse<T><<<(n + 3) / 4, kBlock, 0, str>>>(n, cinv, y, z, st);
    HIPC(hipGetLastError());
}

#define INST_PRE(T, TY) template void vc_pre<T, TY>(const Csr &, const RowCfg &, const T *, const TY *, T *, T *, \
                                                     const PcgState *, hipStream_t);
INST_PRE(double, double)
INST_PRE(float, float)
INST_PRE(float, double)
#define INST_RES(T, TY) template void vc_resid<T, TY>(const Csr &, const RowCfg &, const TY *, const T *, T *, \
                                                       const PcgState *, hipStream_t);
INST_RES(double, double)
INST_RES(float, float)
INST_RES(float, double)
#define INST_POST(T, TY, TZ, D) template void vc_post<T, TY, TZ, D>(const Csr &, const RowCfg &, const T *, const TY *, \
                                                                     const T *, TZ *, double *, unsigned *, PcgState *, hipStream_t);
INST_POST(double, double, double, false)
INST_POST(double, double, double, true)
INST_POST(float, float, float, false)
INST_POST(float, double, float, false)
INST_POST(float, double, double, false)
INST_POST(float, double, double, true)
template void vc_restrict<double>(const Csr &, const RowCfg &, const double *, double *, const PcgState *,
                                  hipStream_t);
template void vc_restrict<float>(const Csr &, const RowCfg &, const float *, float *, const PcgState *, hipStream_t);
template void vc_prolong<double>(const Csr &, const RowCfg &, const double *, double *, const PcgState *,
                                 hipStream_t);
template void vc_prolong<float>(const Csr &, const RowCfg &, const float *, float *, const PcgState *, hipStream_t);
template void coarse_solve<double>(int, const double *, const double *, double *, const PcgState *, hipStream_t);
template void coarse_solve<float>(int, const double *, const float *, float *, const PcgState *, hipStream_t);

void dot_rho(int n, const double *y, const double *z, double *partials, unsigned *counter, PcgState *st,
             hipStream_t s) {
    int g = std::min(kMaxGrid, std::max(1, (n + kBlock - 1) / kBlock));
    k_dot_rho<<<g, kBlock, 0, s>>>(n, y, z, partials, counter, st);
    HIPC(hipGetLastError());
}

void pcg_init(int n, const double *b, double *x, double *r, double *p0, double rtol, double *partials,
              unsigned *counter, PcgState *st, double *hist, hipStream_t s) {
    int g = std::min(kMaxGrid, std::max(8, (n + kBlock - 1) / kBlock));
    k_pcg_init<<<g, kBlock, 0, s>>>(n, b, x, r, p0, rtol, partials, counter, st, hist);
    HIPC(hipGetLastError());
}

void pcg_spmv_p(const Csr &A, const RowCfg &c, const double *z, const double *pold, double *pnew, double *q,
                double *partials, unsigned *counter, PcgState *st, hipStream_t s) {
    const int g = grid_for(A.nr, c), rpb = rows_per_block(A.nr, c, g);
    CAMG_LPR_SWITCH(c.lpr, (k_pcg_spmv_p<L><<<g, kBlock, 0, s>>>(A.nr, rpb, A.rp, A.ci, A.v, z, pold, pnew, q,
                                                                   partials, counter, st)));
    HIPC(hipGetLastError());
}

void pcg_update(int n, const double *p, const double *q, double *x, double *r, double *partials, unsigned *counter,
                PcgState *st, double *hist, int hist_cap, int32_t *hflag, hipStream_t s) {
    int g = std::min(kMaxGrid, std::max(8, (n + kBlock - 1) / kBlock));
    g = (g + 7) / 8 * 8;
    k_pcg_update<<<g, kBlock, 0, s>>>(n, p, q, x, r, partials, counter, st, hist, hist_cap, hflag);
    HIPC(hipGetLastError());
}

void true_residual(const Csr &A, const RowCfg &c, const double *b, const double *x, double *partials,
                   unsigned *counter, double *out2, hipStream_t s) {
    const int g = grid_for(A.nr, c), rpb = rows_per_block(A.nr, c, g);
    CAMG_LPR_SWITCH(c.lpr, (k_true_res<L><<<g, kBlock, 0, s>>>(A.nr, rpb, A.rp, A.ci, A.v, b, x, partials, counter,
                                                                 out2)));
    HIPC(hipGetLastError());
}

void fill_zero(int64_t n, double *x, hipStream_t s) {
    if (n > 0) k_fill_zero<<<(int)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, x);
    HIPC(hipGetLastError());
}

}  // namespace camg
