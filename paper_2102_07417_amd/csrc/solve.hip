// Solve-phase kernels: the V-cycle of Alg. "AMG application in a V-cycle"
// with Jacobi smoothing (eq. smoother, M = D) and the PCG recurrence.
//
// Row kernels come in two shapes, chosen per matrix at set-up:
//  - tile: a block takes `rpt` consecutive rows whose nonzeros fit an LDS
//    tile; phase 1 streams the tile's column indices and values with
//    coalesced loads, forms a_ij * g(x_j) for every nonzero (many gathers in
//    flight per thread) and parks the products in LDS; phase 2 lets `lpr`
//    lanes per row add them up and runs the row's epilogue.  Used whenever
//    the longest row fits the tile (every matrix of the workloads here).
//  - vector: `lpr` lanes walk each row directly (rows too long for a tile).
// Blocks are renumbered so that each XCD owns one contiguous slab of rows
// (its L2 then serves the gathered vector entries those rows share).
//
// Reductions are deterministic and fence-free: a producing kernel writes one
// partial per block; the consuming kernel (one kernel later in the stream)
// adds the partials in index order in every block that needs the total.
// Scalars of the recurrence stay in device memory; once the stopping test
// passes, every later kernel sees `done` and returns at once.
#include "devutil.hpp"
#include "internal.hpp"

namespace camg {

namespace {

constexpr int kTileNnz = 2048;  // LDS tile capacity (nonzeros)

template <class T>
struct MatArg {
    const int32_t *__restrict__ rp;
    const int32_t *__restrict__ ci;
    const T *__restrict__ v;
    int n;
    int rpt;     // tile: rows per tile; vector: rows per block
    int ntiles;  // tile mode
    int tpb;     // tiles per block
};

template <class T>
static const T *vals(const Csr &A);
template <>
const double *vals<double>(const Csr &A) { return A.v; }
template <>
const float *vals<float>(const Csr &A) { return A.v32; }

template <class T>
MatArg<T> mat_arg(const Csr &A, const RowCfg &c) {
    return MatArg<T>{A.rp, A.ci, vals<T>(A), A.nr, c.rpt, c.ntiles, c.tpb};
}

// Sum of partials[0..n) in index order, result in every thread of the block.
__device__ __forceinline__ double sum_all(const double *partials, int n) {
    __shared__ double tot;
    const double t = sum_partials<kBlock>(partials, n);
    if (threadIdx.x == 0) tot = t;
    __syncthreads();
    const double r = tot;
    __syncthreads();
    return r;
}

// Walk this block's rows; for each row call epi(i, sum_j a_ij g(j), dot).
template <class T, int LPR, bool TILE, class G, class E>
__device__ __forceinline__ void run_rows(const MatArg<T> &M, const G &g, const E &epi, T *prod, double &dot) {
    const int sl = threadIdx.x & (LPR - 1), grp = threadIdx.x / LPR;
    constexpr int RPP = kBlock / LPR;  // rows per pass
    if (TILE) {
        const int b = xcd_block();
        const int t0 = b * M.tpb, t1 = min(M.ntiles, t0 + M.tpb);
        for (int t = t0; t < t1; ++t) {
            const int r0 = t * M.rpt, r1 = min(M.n, r0 + M.rpt);
            const int e0 = M.rp[r0], m = M.rp[r1] - e0;
            int k = threadIdx.x;
            for (; k + 3 * kBlock < m; k += 4 * kBlock) {
                const int e = e0 + k;
                const int j0 = M.ci[e], j1 = M.ci[e + kBlock], j2 = M.ci[e + 2 * kBlock], j3 = M.ci[e + 3 * kBlock];
                const T a0 = M.v[e], a1 = M.v[e + kBlock], a2 = M.v[e + 2 * kBlock], a3 = M.v[e + 3 * kBlock];
                const T g0 = g(j0), g1 = g(j1), g2 = g(j2), g3 = g(j3);
                prod[k] = a0 * g0;
                prod[k + kBlock] = a1 * g1;
                prod[k + 2 * kBlock] = a2 * g2;
                prod[k + 3 * kBlock] = a3 * g3;
            }
            for (; k < m; k += kBlock) {
                const int e = e0 + k;
                prod[k] = M.v[e] * g(M.ci[e]);
            }
            __syncthreads();
            for (int ib = r0; ib < r1; ib += RPP) {
                const int i = ib + grp;
                T acc = 0;
                if (i < r1) {
                    const int a = M.rp[i] - e0, z = M.rp[i + 1] - e0;
                    for (int q = a + sl; q < z; q += LPR) acc += prod[q];
                }
                acc = group_sum<LPR>(acc);
                if (i < r1 && sl == 0) epi(i, acc, dot);
            }
            __syncthreads();
        }
    } else {
        const int b = xcd_block();
        const int r0 = min(M.n, b * M.rpt), r1 = min(M.n, r0 + M.rpt);
        for (int ib = r0; ib < r1; ib += RPP) {
            const int i = ib + grp;
            T acc = 0;
            if (i < r1) {
                const int e1 = M.rp[i + 1];
                for (int e = M.rp[i] + sl; e < e1; e += LPR) acc += M.v[e] * g(M.ci[e]);
            }
            acc = group_sum<LPR>(acc);
            if (i < r1 && sl == 0) epi(i, acc, dot);
        }
    }
}

// ------------------------------------------------------------------ gathers and epilogues
template <class T, class TY>
struct GPre {  // s_j of the first Jacobi step from s = 0
    const T *wd;
    const TY *y;
    __device__ T operator()(int j) const { return wd[j] * (T)y[j]; }
};
template <class T>
struct GVec {
    const T *x;
    __device__ T operator()(int j) const { return x[j]; }
};
struct GDir {  // the new search direction, formed on the fly
    const double *z, *p;
    double beta;
    bool first;
    __device__ double operator()(int j) const { return first ? z[j] : z[j] + beta * p[j]; }
};

template <class T, class TY>
struct EPre {  // s = wd y, r = y - A s
    const T *wd;
    const TY *y;
    T *s, *r;
    __device__ void operator()(int i, T acc, double &) const {
        const T yi = (T)y[i];
        s[i] = wd[i] * yi;
        r[i] = yi - acc;
    }
};
template <class T, class TY, class TZ>
struct EPost {  // z = s + wd (y - A s); dot += y.z
    const T *wd;
    const TY *y;
    const T *s;
    TZ *z;
    __device__ void operator()(int i, T acc, double &dot) const {
        const T yi = (T)y[i];
        const T zi = s[i] + wd[i] * (yi - acc);
        const TZ zo = (TZ)zi;
        z[i] = zo;
        dot += (double)y[i] * (double)zo;
    }
};
template <class T, class TY>
struct EResid {  // r = y - A s
    const TY *y;
    T *r;
    __device__ void operator()(int i, T acc, double &) const { r[i] = (T)y[i] - acc; }
};
template <class T, bool ADD>
struct ESpmv {
    T *out;
    __device__ void operator()(int i, T acc, double &) const { out[i] = ADD ? out[i] + acc : acc; }
};
struct EDir {  // p_new, q = A p_new, dot += p.q
    const double *z, *pold;
    double beta;
    bool first;
    double *pnew, *q;
    __device__ void operator()(int i, double acc, double &dot) const {
        const double pi = first ? z[i] : z[i] + beta * pold[i];
        pnew[i] = pi;
        q[i] = acc;
        dot += pi * acc;
    }
};
struct EResNorm {  // d = b - A x; dot += d^2; optionally store d
    const double *b;
    double *out;
    __device__ void operator()(int i, double acc, double &dot) const {
        const double d = b[i] - acc;
        if (out) out[i] = d;
        dot += d * d;
    }
};

// ------------------------------------------------------------------ kernels
template <class T, int LPR, bool TILE, bool DOT, class G, class E>
__global__ void __launch_bounds__(kBlock) k_rows(MatArg<T> M, G g, E e, double *partials, const PcgState *st) {
    if (st && st->done) return;
    extern __shared__ double smem_d[];
    T *prod = reinterpret_cast<T *>(smem_d);
    double dot = 0.0;
    run_rows<T, LPR, TILE>(M, g, e, prod, dot);
    if (DOT) {
        const double b = block_sum<kBlock>(dot);
        if (threadIdx.x == 0) partials[blockIdx.x] = b;
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

// partial sums of y.z (one-level hierarchy: nothing to fuse into)
__global__ void __launch_bounds__(kBlock) k_dot(int n, const double *__restrict__ y, const double *__restrict__ z,
                                                double *partials, const PcgState *st) {
    if (st && st->done) return;
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) acc += y[i] * z[i];
    const double b = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// x = 0, r = b, p = 0; partials of ||b||^2; state reset
__global__ void __launch_bounds__(kBlock) k_pcg_init(int n, const double *__restrict__ b, double *__restrict__ x,
                                                     double *__restrict__ r, double *__restrict__ p0, double rtol,
                                                     double *pr2, PcgState *st) {
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
    if (threadIdx.x == 0) {
        pr2[blockIdx.x] = bs;
        if (blockIdx.x == 0) {
            st->rho = st->rho_old = st->sigma = st->alpha = st->beta = 0.0;
            st->rnorm = 0.0;
            st->bnorm = -1.0;
            st->tol = -1.0;
            st->rtol = rtol;
            st->iter = 0;
            st->done = 0;
            st->status = 0;
            st->restart = 0;
        }
    }
}

// Stopping test at the start of an iteration (and once after the last):
// ||r_k|| from the partials of the kernel that formed r_k.
__global__ void __launch_bounds__(kBlock) k_pcg_check(const double *pr2, int npr2, PcgState *st, double *hist,
                                                      int hist_cap, int32_t *hflag) {
    if (st->done) return;
    const double rn = sqrt(sum_all(pr2, npr2));
    if (threadIdx.x == 0) {
        if (st->bnorm < 0.0) {
            st->bnorm = rn;
            st->tol = st->rtol > 0.0 ? st->rtol * rn : -1.0;
        }
        const int it = st->iter;
        if (it < hist_cap) hist[it] = rn;
        st->rnorm = rn;
        if (st->bnorm == 0.0 || (st->tol > 0.0 && rn < st->tol)) {
            st->done = 1;
            if (hflag) hflag[0] = 1;
        }
    }
}

// rho = sum of the post-smoothing partials; p_new = z + beta p_old;
// q = A p_new; partials of p_new . q
template <int LPR, bool TILE>
__global__ void __launch_bounds__(kBlock) k_pcg_dir(MatArg<double> M, const double *__restrict__ z,
                                                    const double *__restrict__ pold, double *__restrict__ pnew,
                                                    double *__restrict__ q, const double *prz, int nprz, double *ppq,
                                                    PcgState *st) {
    if (st->done) return;
    extern __shared__ double smem_d[];
    const double rho = sum_all(prz, nprz);
    const bool first = st->iter == st->restart;
    const double beta = first ? 0.0 : rho / st->rho_old;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho = rho;
        st->beta = beta;
    }
    double dot = 0.0;
    run_rows<double, LPR, TILE>(M, GDir{z, pold, beta, first}, EDir{z, pold, beta, first, pnew, q}, smem_d, dot);
    const double b = block_sum<kBlock>(dot);
    if (threadIdx.x == 0) ppq[blockIdx.x] = b;
}

// sigma = sum of the p.q partials; breakdown test; alpha = rho / sigma;
// x += alpha p, r -= alpha q; partials of ||r||^2
__global__ void __launch_bounds__(kBlock) k_pcg_update(int n, const double *__restrict__ p,
                                                       const double *__restrict__ q, double *__restrict__ x,
                                                       double *__restrict__ r, const double *ppq, int nppq,
                                                       double *pr2, PcgState *st, int32_t *hflag) {
    if (st->done) return;
    const double sigma = sum_all(ppq, nppq);
    const double rho = st->rho;
    if (!(sigma > 0.0) || !(rho > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->sigma = sigma;
            st->status = (int32_t)CAMG_E_BREAKDOWN;
            st->done = 1;
            if (hflag) hflag[0] = 1;
        }
        return;
    }
    const double alpha = rho / sigma;
    double acc = 0.0;
    const int stride = gridDim.x * kBlock;
    for (int i = xcd_block() * kBlock + threadIdx.x; i < n; i += stride) {
        x[i] = x[i] + alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    const double bs = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) {
        pr2[blockIdx.x] = bs;
        if (blockIdx.x == 0) {
            st->sigma = sigma;
            st->alpha = alpha;
            st->rho_old = rho;
            st->iter = st->iter + 1;
        }
    }
}

// after a residual replacement: restart the recurrence at the current iterate
__global__ void k_pcg_restart(PcgState *st) {
    st->done = 0;
    st->status = 0;
    st->restart = st->iter;
}

__global__ void __launch_bounds__(kBlock) k_sum_to(const double *partials, int n, double *out) {
    const double t = sum_partials<kBlock>(partials, n);
    if (threadIdx.x == 0) *out = t;
}

// ------------------------------------------------------------------ dispatch
#define CAMG_LPR_SWITCH(lpr, ...)                          \
    switch (lpr) {                                         \
    case 1: { constexpr int L = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int L = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int L = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int L = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int L = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int L = 32; __VA_ARGS__; } break; \
    default: { constexpr int L = 64; __VA_ARGS__; } break; \
    }

template <class T, bool DOT, class G, class E>
void launch_rows(const Csr &A, const RowCfg &c, const G &g, const E &e, double *partials, const PcgState *st,
                 hipStream_t s) {
    const MatArg<T> M = mat_arg<T>(A, c);
    const size_t smem = c.tile ? (size_t)c.tile_nnz * sizeof(T) : 0;
    if (c.tile) {
        CAMG_LPR_SWITCH(c.lpr, (k_rows<T, L, true, DOT, G, E><<<c.grid, kBlock, smem, s>>>(M, g, e, partials, st)));
    } else {
        CAMG_LPR_SWITCH(c.lpr, (k_rows<T, L, false, DOT, G, E><<<c.grid, kBlock, 0, s>>>(M, g, e, partials, st)));
    }
    HIPC(hipGetLastError());
}

int pow2_ceil(double x) {
    int p = 1;
    while (p < x && p < 64) p <<= 1;
    return p;
}

}  // namespace

RowCfg choose_cfg(int n, int64_t nnz, int maxrow) {
    RowCfg c;
    const double mean = n > 0 ? (double)nnz / n : 1.0;
    if (maxrow <= kTileNnz) {
        c.tile = true;
        int rpt = 1;
        while (rpt * 2 <= 1024 && (int64_t)rpt * 2 * std::max(maxrow, 1) <= kTileNnz) rpt *= 2;
        c.rpt = rpt;
        c.tile_nnz = rpt * std::max(maxrow, 1);
        c.lpr = std::max(1, pow2_ceil(mean) / 2);
        c.ntiles = (n + rpt - 1) / rpt;
        int g = std::min(c.ntiles, kMaxGrid);
        g = std::max(8, (g + 7) / 8 * 8);
        c.grid = g;
        c.tpb = (c.ntiles + g - 1) / g;
    } else {
        c.tile = false;
        c.lpr = 64;
        const int rpp = kBlock / c.lpr;
        int g = (n + rpp - 1) / rpp;
        g = std::min(g, kMaxGrid);
        g = std::max(8, (g + 7) / 8 * 8);
        c.grid = g;
        const int per = (n + g - 1) / g;
        c.rpt = (per + rpp - 1) / rpp * rpp;
        c.ntiles = 0;
        c.tpb = 0;
        c.tile_nnz = 0;
    }
    c.maxrow = maxrow;
    return c;
}

int vec_grid(int n) {
    int g = std::min(kMaxGrid, std::max(8, (n + kBlock - 1) / kBlock));
    return (g + 7) / 8 * 8;
}

template <class T, class TY>
void vc_pre(const Csr &A, const RowCfg &c, const T *wd, const TY *y, T *s, T *r, const PcgState *st,
            hipStream_t str) {
    launch_rows<T, false>(A, c, GPre<T, TY>{wd, y}, EPre<T, TY>{wd, y, s, r}, nullptr, st, str);
}

template <class T, class TY, class TZ, bool DOT>
void vc_post(const Csr &A, const RowCfg &c, const T *wd, const TY *y, const T *s, TZ *z, double *partials,
             const PcgState *st, hipStream_t str) {
    launch_rows<T, DOT>(A, c, GVec<T>{s}, EPost<T, TY, TZ>{wd, y, s, z}, partials, st, str);
}

template <class T, class TY>
void vc_resid(const Csr &A, const RowCfg &c, const TY *y, const T *s, T *r, const PcgState *st, hipStream_t str) {
    launch_rows<T, false>(A, c, GVec<T>{s}, EResid<T, TY>{y, r}, nullptr, st, str);
}

template <class T>
void vc_restrict(const Csr &R, const RowCfg &c, const T *r, T *yc, const PcgState *st, hipStream_t str) {
    launch_rows<T, false>(R, c, GVec<T>{r}, ESpmv<T, false>{yc}, nullptr, st, str);
}

template <class T>
void vc_prolong(const Csr &P, const RowCfg &c, const T *d, T *s, const PcgState *st, hipStream_t str) {
    launch_rows<T, false>(P, c, GVec<T>{d}, ESpmv<T, true>{s}, nullptr, st, str);
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
                                                                     const T *, TZ *, double *, const PcgState *, hipStream_t);
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

int dot_partials(int n, const double *y, const double *z, double *partials, const PcgState *st, hipStream_t s) {
    const int g = std::min(kMaxGrid, std::max(1, (n + kBlock - 1) / kBlock));
    k_dot<<<g, kBlock, 0, s>>>(n, y, z, partials, st);
    HIPC(hipGetLastError());
    return g;
}

int pcg_init(int n, const double *b, double *x, double *r, double *p0, double rtol, double *pr2, PcgState *st,
             hipStream_t s) {
    const int g = vec_grid(n);
    k_pcg_init<<<g, kBlock, 0, s>>>(n, b, x, r, p0, rtol, pr2, st);
    HIPC(hipGetLastError());
    return g;
}

void pcg_check(const double *pr2, int npr2, PcgState *st, double *hist, int hist_cap, int32_t *hflag, hipStream_t s) {
    k_pcg_check<<<1, kBlock, 0, s>>>(pr2, npr2, st, hist, hist_cap, hflag);
    HIPC(hipGetLastError());
}

int pcg_dir(const Csr &A, const RowCfg &c, const double *z, const double *pold, double *pnew, double *q,
            const double *prz, int nprz, double *ppq, PcgState *st, hipStream_t s) {
    const MatArg<double> M = mat_arg<double>(A, c);
    const size_t smem = c.tile ? (size_t)c.tile_nnz * sizeof(double) : 0;
    if (c.tile) {
        CAMG_LPR_SWITCH(c.lpr, (k_pcg_dir<L, true><<<c.grid, kBlock, smem, s>>>(M, z, pold, pnew, q, prz, nprz, ppq, st)));
    } else {
        CAMG_LPR_SWITCH(c.lpr, (k_pcg_dir<L, false><<<c.grid, kBlock, 0, s>>>(M, z, pold, pnew, q, prz, nprz, ppq, st)));
    }
    HIPC(hipGetLastError());
    return c.grid;
}

int pcg_update(int n, const double *p, const double *q, double *x, double *r, const double *ppq, int nppq, double *pr2,
               PcgState *st, int32_t *hflag, hipStream_t s) {
    const int g = vec_grid(n);
    k_pcg_update<<<g, kBlock, 0, s>>>(n, p, q, x, r, ppq, nppq, pr2, st, hflag);
    HIPC(hipGetLastError());
    return g;
}

void pcg_restart(PcgState *st, hipStream_t s) {
    k_pcg_restart<<<1, 1, 0, s>>>(st);
    HIPC(hipGetLastError());
}

int residual_norm(const Csr &A, const RowCfg &c, const double *b, const double *x, double *out, double *partials,
                  hipStream_t s) {
    launch_rows<double, true>(A, c, GVec<double>{x}, EResNorm{b, out}, partials, nullptr, s);
    return c.grid;
}

void sum_to(const double *partials, int n, double *out, hipStream_t s) {
    k_sum_to<<<1, kBlock, 0, s>>>(partials, n, out);
    HIPC(hipGetLastError());
}

}  // namespace camg
