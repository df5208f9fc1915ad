// Many right-hand sides at once: k independent PCG recurrences that share
// every matrix pass.  The vectors are row-major n-by-K blocks (K = the
// engine's slot count, a power of two up to 64), so the K values of one row
// are contiguous: a gather of row j of the block is one coalesced segment
// and every matrix entry is read once for all K columns.
//
// Row kernels put K lanes on a row, lane c owning column c; the group loads
// up to K nonzeros of the row cooperatively and broadcasts them with
// shuffles, and each lane adds its column's products in CSR order.  Each
// column's arithmetic therefore does not depend on the other columns, on how
// many are in use or on which slot it occupies, and the per-column dot
// products are summed over a fixed row partition in a fixed order: a
// column's iterates are bitwise the same alone and inside any batch on an
// engine with the same slot count.
//
// Per-column state (rho, alpha, beta, iteration count, done flag, ...) lives
// in device memory; a finished column stops updating while the others go on,
// and a free slot can be started while the others run (the serving loop
// uses that for continuous batching).
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <memory>
#include <vector>

#include "devutil.hpp"
#include "internal.hpp"

namespace camg {

namespace {

struct MState;
}  // namespace
struct Engine;
namespace {

constexpr int kRed = 1024;       // threads of the one-block reductions
constexpr int kMGridMax = 2048;  // most blocks of a block-row kernel (partials per column)

struct MState {
    double rho[kMaxSlots], rho_old[kMaxSlots], sigma[kMaxSlots], alpha[kMaxSlots], beta[kMaxSlots];
    double rnorm[kMaxSlots], bnorm[kMaxSlots], tol[kMaxSlots], rtol[kMaxSlots];
    int32_t iter[kMaxSlots], done[kMaxSlots], status[kMaxSlots], restart[kMaxSlots], active[kMaxSlots];
    int32_t max_iter[kMaxSlots];
    int32_t running;  // columns active and not done, as of the last stopping test
    int32_t pad;
};

__device__ __forceinline__ bool running(const MState *st, int c) { return st->active[c] && !st->done[c]; }

// Balanced contiguous row range of this block (blocks renumbered per XCD).
__device__ __forceinline__ void block_rows(int n, int &r0, int &r1) {
    const int b = xcd_block();
    r0 = (int)((int64_t)b * n / gridDim.x);
    r1 = (int)((int64_t)(b + 1) * n / gridDim.x);
}

// Per-column sums over the block: lanes with the same column add their
// values in group order; partials[blockIdx.x * K + c].
template <int K>
__device__ __forceinline__ void block_col_sum(double v, double *partials, unsigned long long mask = ~0ull) {
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < K && ((mask >> threadIdx.x) & 1ull)) {
        double t = 0.0;
        for (int g = 0; g < kBlock / K; ++g) t += sh[g * K + threadIdx.x];
        partials[(size_t)blockIdx.x * K + threadIdx.x] = t;
    }
    __syncthreads();
}

// Sum over blocks of partials[b * K + c] for every column, by one block of
// kRed threads; result of column c in out[c] (shared).  Fixed order: thread
// (g, c) adds blocks g, g + per, ... into four running sums, then the per
// group sums are added pairwise in a fixed tree.
template <int K>
__device__ __forceinline__ void sum_cols(const double *partials, int nb, double *out) {
    __shared__ double sh[kRed];
    constexpr int per = kRed / K;
    const int c = threadIdx.x % K, g = threadIdx.x / K;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
    int b = g;
    for (; b + 3 * per < nb; b += 4 * per) {
        t0 += partials[(size_t)b * K + c];
        t1 += partials[(size_t)(b + per) * K + c];
        t2 += partials[(size_t)(b + 2 * per) * K + c];
        t3 += partials[(size_t)(b + 3 * per) * K + c];
    }
    for (; b < nb; b += per) t0 += partials[(size_t)b * K + c];
    sh[threadIdx.x] = (t0 + t1) + (t2 + t3);
    __syncthreads();
    for (int s = per / 2; s >= 1; s >>= 1) {
        if (g < s) sh[threadIdx.x] += sh[threadIdx.x + s * K];
        __syncthreads();
    }
    if (threadIdx.x < K) out[threadIdx.x] = sh[threadIdx.x];
    __syncthreads();
}

// ------------------------------------------------------------------ row kernel
// out(i, c) = sum_j a_ij g(j, c); epi(i, c, acc, dot).  The row's entries
// are taken eight at a time: the lanes of a group read the same index and
// value (one cache line per group), clamped to the row so every load and
// gather is unconditional and all are in flight together; the products are
// added in CSR order, the padding ones skipped.
template <class T, int K, bool DOT, class G, class E>
__global__ void __launch_bounds__(kBlock) mk_rows(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                  const T *__restrict__ av, G g, E epi, double *partials,
                                                  unsigned long long pmask) {
    constexpr int RPP = kBlock / K;
    constexpr int U = 8;
    const int c = threadIdx.x % K, grp = threadIdx.x / K;
    int r0, r1;
    block_rows(n, r0, r1);
    double dot = 0.0;
    for (int i = r0 + grp; i < r1; i += RPP) {
        const int e0 = rp[i], e1 = rp[i + 1];
        T acc = 0;
        for (int eb = e0; eb < e1; eb += U) {
            int j[U];
            T a[U], x[U];
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const int e = min(eb + t, e1 - 1);
                j[t] = ci[e];
                a[t] = av[e];
            }
#pragma unroll
            for (int t = 0; t < U; ++t) x[t] = g(j[t], c);
#pragma unroll
            for (int t = 0; t < U; ++t)
                if (eb + t < e1) acc += a[t] * x[t];
        }
        epi(i, c, acc, dot);
    }
    if (DOT) block_col_sum<K>(dot, partials, pmask);
}

template <class T, int K, class TX = T>
struct MGather {
    const TX *x;
    __device__ T operator()(int j, int c) const { return (T)x[(size_t)j * K + c]; }
};

template <class T, int K, class TY>
struct MEPre {  // S = wd Y, R = Y - (A wd) Y  (values pre-scaled by wd)
    const T *wd;
    const TY *y;
    T *s, *r;
    __device__ void operator()(int i, int c, T acc, double &) const {
        const size_t o = (size_t)i * K + c;
        const T yi = (T)y[o];
        s[o] = wd[i] * yi;
        r[o] = yi - acc;
    }
};
template <class T, int K, class TY, class TZ>
struct MEPost {  // Z = S + wd (Y - A S); dot += Y Z
    const T *wd;
    const TY *y;
    const T *s;
    TZ *z;
    __device__ void operator()(int i, int c, T acc, double &dot) const {
        const size_t o = (size_t)i * K + c;
        const T zi = s[o] + wd[i] * ((T)y[o] - acc);
        const TZ zo = (TZ)zi;
        z[o] = zo;
        dot += (double)y[o] * (double)zo;
    }
};
template <class T, int K, class TY>
struct MEResid {
    const TY *y;
    T *r;
    __device__ void operator()(int i, int c, T acc, double &) const {
        const size_t o = (size_t)i * K + c;
        r[o] = (T)y[o] - acc;
    }
};
template <class T, int K, bool ADD>
struct MESpmv {
    T *out;
    __device__ void operator()(int i, int c, T acc, double &) const {
        const size_t o = (size_t)i * K + c;
        out[o] = ADD ? out[o] + acc : acc;
    }
};
template <int K>
struct MGDir {  // P_new = Z + beta_c P_old, on the fly
    const double *z, *p;
    const double *beta;
    __device__ double operator()(int j, int c) const {
        const size_t o = (size_t)j * K + c;
        return z[o] + beta[c] * p[o];
    }
};
template <int K>
struct MEDir {
    const double *z, *pold;
    const double *beta;
    double *pnew, *q;
    __device__ void operator()(int i, int c, double acc, double &dot) const {
        const size_t o = (size_t)i * K + c;
        const double pi = z[o] + beta[c] * pold[o];
        pnew[o] = pi;
        q[o] = acc;
        dot += pi * acc;
    }
};
template <int K>
struct MERes {  // d = B - A X; dot += d^2; R = d for the columns of `mask`
    const double *b;
    double *out;
    unsigned long long mask;
    __device__ void operator()(int i, int c, double acc, double &dot) const {
        const size_t o = (size_t)i * K + c;
        const double d = b[o] - acc;
        if (out && ((mask >> c) & 1ull)) out[o] = d;
        dot += d * d;
    }
};

// ------------------------------------------------------------------ elementwise / state kernels
// Start the columns c with q.q[c] >= 0 from column q.q[c] of B (n-by-m
// row-major, row stride ldb): X = 0, R = B, both P = 0; state reset;
// partials of ||b||^2 for them.
template <int K>
__global__ void __launch_bounds__(kBlock) mk_start(int n, SlotMap q, const double *__restrict__ B, int ldb,
                                                   double *X, double *R, double *B0, double *P0, double *P1,
                                                   double rtol, int max_iter, double *pr2, MState *st) {
    constexpr int RPP = kBlock / K;
    const int c = threadIdx.x % K, grp = threadIdx.x / K;
    const int qc = q.q[c];
    const bool mine = qc >= 0;
    int r0, r1;
    block_rows(n, r0, r1);
    double acc = 0.0;
    if (mine)
        for (int i = r0 + grp; i < r1; i += RPP) {
            const size_t o = (size_t)i * K + c;
            const double bi = B[(size_t)i * ldb + qc];
            X[o] = 0.0;
            R[o] = bi;
            B0[o] = bi;
            P0[o] = 0.0;
            P1[o] = 0.0;
            acc += bi * bi;
        }
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < K && mine) {
        double t = 0.0;
        for (int g = 0; g < RPP; ++g) t += sh[g * K + threadIdx.x];
        pr2[(size_t)blockIdx.x * K + threadIdx.x] = t;
        if (blockIdx.x == 0) {
            st->rho[c] = st->rho_old[c] = st->sigma[c] = st->alpha[c] = st->beta[c] = 0.0;
            st->rnorm[c] = 0.0;
            st->bnorm[c] = -1.0;
            st->tol[c] = -1.0;
            st->rtol[c] = rtol;
            st->iter[c] = 0;
            st->done[c] = 0;
            st->status[c] = 0;
            st->restart[c] = 0;
            st->active[c] = 1;
            st->max_iter[c] = max_iter;
        }
    }
}

// free the slots of `mask`
template <int K>
__global__ void mk_release(MState *st, unsigned long long mask) {
    const int c = threadIdx.x;
    if (c < K && ((mask >> c) & 1ull)) st->active[c] = 0;
}

// per-column state (and, when sq is given, the true ||b - A x||^2 sums)
// into a plain snapshot for the host
template <int K>
__global__ void mk_snap(const MState *st, const double *sq, EngineSnap *out) {
    const int c = threadIdx.x;
    if (c < K) {
        out->iter[c] = st->iter[c];
        out->done[c] = st->done[c];
        out->status[c] = st->status[c];
        out->active[c] = st->active[c];
        out->rnorm[c] = st->rnorm[c];
        out->bnorm[c] = st->bnorm[c];
        out->tres2[c] = sq ? sq[c] : -1.0;
    }
}

// out (n-by-k row-major) = the columns q.q[0..k) of X
template <int K>
__global__ void __launch_bounds__(kBlock) mk_gather_cols(int n, int k, SlotMap q, const double *__restrict__ X,
                                                         double *__restrict__ out) {
    const int64_t tot = (int64_t)n * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / k;
        const int j = (int)(t - i * k);
        out[t] = X[i * K + q.q[j]];
    }
}

// Stopping test of every running column (one block); hist is K-by-cap.
template <int K>
__global__ void __launch_bounds__(kRed) mk_check(const double *pr2, int nb, MState *st, double *hist, int cap,
                                                   int32_t *hflag) {
    __shared__ double tot[K];
    sum_cols<K>(pr2, nb, tot);
    if (threadIdx.x < K) {
        const int c = threadIdx.x;
        if (running(st, c)) {
            const double rn = sqrt(tot[c]);
            if (st->bnorm[c] < 0.0) {
                st->bnorm[c] = rn;
                st->tol[c] = st->rtol[c] > 0.0 ? st->rtol[c] * rn : -1.0;
            }
            const int it = st->iter[c];
            if (hist && it < cap) hist[(size_t)c * cap + it] = rn;
            st->rnorm[c] = rn;
            if (st->bnorm[c] == 0.0 || (st->tol[c] > 0.0 && rn < st->tol[c])) {
                st->done[c] = 1;
            } else if (it >= st->max_iter[c]) {
                st->done[c] = 1;
                st->status[c] = (int32_t)CAMG_E_MAXIT;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        for (int c = 0; c < K; ++c) r += running(st, c) ? 1 : 0;
        st->running = r;
        if (hflag) hflag[0] = r;
    }
}

// rho_c and beta_c of every running column (one block)
template <int K>
__global__ void __launch_bounds__(kRed) mk_fin_rz(const double *prz, int nb, MState *st) {
    __shared__ double tot[K];
    sum_cols<K>(prz, nb, tot);
    if (threadIdx.x < K) {
        const int c = threadIdx.x;
        double beta = 0.0;
        if (running(st, c)) {
            const double rho = tot[c];
            st->rho[c] = rho;
            if (st->iter[c] != st->restart[c]) beta = rho / st->rho_old[c];
        }
        st->beta[c] = beta;
    }
}

// sigma_c, breakdown test, alpha_c; iteration count (one block)
template <int K>
__global__ void __launch_bounds__(kRed) mk_fin_pq(const double *ppq, int nb, MState *st) {
    __shared__ double tot[K];
    sum_cols<K>(ppq, nb, tot);
    if (threadIdx.x < K) {
        const int c = threadIdx.x;
        double alpha = 0.0;
        if (running(st, c)) {
            const double sigma = tot[c], rho = st->rho[c];
            st->sigma[c] = sigma;
            if (!(sigma > 0.0) || !(rho > 0.0)) {
                st->done[c] = 1;
                st->status[c] = (int32_t)CAMG_E_BREAKDOWN;
            } else {
                alpha = rho / sigma;
                st->rho_old[c] = rho;
                st->iter[c] += 1;
            }
        }
        st->alpha[c] = alpha;
    }
}

// X += alpha P, R -= alpha Q for running columns; partials of ||R||^2
template <int K>
__global__ void __launch_bounds__(kBlock) mk_update(int n, const double *__restrict__ P, const double *__restrict__ Q,
                                                    double *X, double *R, double *pr2, const MState *st) {
    constexpr int RPP = kBlock / K;
    const int c = threadIdx.x % K, grp = threadIdx.x / K;
    int r0, r1;
    block_rows(n, r0, r1);
    const bool run = st->alpha[c] != 0.0;
    const double a = st->alpha[c];
    double acc = 0.0;
    for (int i = r0 + grp; i < r1; i += RPP) {
        const size_t o = (size_t)i * K + c;
        double ri = R[o];
        if (run) {
            X[o] = X[o] + a * P[o];
            ri = ri - a * Q[o];
            R[o] = ri;
        }
        acc += ri * ri;
    }
    block_col_sum<K>(acc, pr2);
}

// partials of the per-column dot products Y.Z
template <int K>
__global__ void __launch_bounds__(kBlock) mk_dot(int n, const double *__restrict__ Y, const double *__restrict__ Z,
                                                 double *partials) {
    constexpr int RPP = kBlock / K;
    const int c = threadIdx.x % K, grp = threadIdx.x / K;
    int r0, r1;
    block_rows(n, r0, r1);
    double acc = 0.0;
    for (int i = r0 + grp; i < r1; i += RPP) acc += Y[(size_t)i * K + c] * Z[(size_t)i * K + c];
    block_col_sum<K>(acc, partials);
}

// restart columns whose true residual failed the test after a replacement
template <int K>
__global__ void mk_restart(MState *st, unsigned long long mask) {
    const int c = threadIdx.x;
    if (c < K && ((mask >> c) & 1ull)) {
        st->done[c] = 0;
        st->status[c] = 0;
        st->restart[c] = st->iter[c];
    }
}

template <int K>
__global__ void __launch_bounds__(kRed) mk_sum(const double *partials, int nb, double *out) {
    __shared__ double tot[K];
    sum_cols<K>(partials, nb, tot);
    if (threadIdx.x < K) out[threadIdx.x] = tot[threadIdx.x];
}

// last level: Z = Ainv Y for a K-column block (FP64 arithmetic), K lanes
// per row; eight loads in flight, products added in column order
template <class T, int K>
__global__ void __launch_bounds__(kBlock) mk_coarse(int n, const double *__restrict__ cinv, const T *__restrict__ y,
                                                    T *__restrict__ z) {
    constexpr int RPP = kBlock / K;
    const int c = threadIdx.x % K;
    const int i = blockIdx.x * RPP + threadIdx.x / K;
    if (i >= n) return;
    const double *row = cinv + (size_t)i * n;
    double acc = 0.0;
    int j = 0;
    for (; j + 8 <= n; j += 8) {
        double a[8], v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            a[t] = row[j + t];
            v[t] = (double)y[(size_t)(j + t) * K + c];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) acc += a[t] * v[t];
    }
    for (; j < n; ++j) acc += row[j] * (double)y[(size_t)j * K + c];
    z[(size_t)i * K + c] = (T)acc;
}

int mgrid(int n, int K) {
    const int rpp = kBlock / K;
    int g = (n + rpp - 1) / rpp;
    g = std::min(g, kMGridMax);
    return std::max(8, (g + 7) / 8 * 8);
}

}  // namespace

// ======================================================================= engine
struct Engine {
    Hier *h = nullptr;
    int K = 0;
    int n = 0;
    bool mixed = false;
    Pool pool;
    double *X = nullptr, *R = nullptr, *Bk = nullptr, *Z = nullptr, *P[2] = {nullptr, nullptr}, *Q = nullptr;
    struct Lv {
        void *y = nullptr, *s = nullptr, *r = nullptr, *z = nullptr, *t = nullptr;
        int grid = 8;   // row-kernel grid of A_l
        int gridP = 8, gridR = 8;
    };
    std::vector<Lv> lv;
    double *pr2 = nullptr, *prz = nullptr, *ppq = nullptr, *ptmp = nullptr, *sc = nullptr;
    int nb_vec = 8;     // blocks of the n-row elementwise kernels
    MState *st = nullptr;
    double *hist = nullptr;
    int cap = 0;
    int32_t *hflag = nullptr, *hflag_dev = nullptr;
    hipStream_t stream = nullptr;
    int par = 0;        // parity of the next iteration
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    bool graph_ok = false;
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    ~Engine();
};

namespace {

template <class T, int K, class G, class Ep>
void launch_mrows_any(int n, const int32_t *rp, const int32_t *ci, const T *av, int grid, hipStream_t s,
                      const G &g, const Ep &e, double *partials, bool dot, unsigned long long pmask = ~0ull) {
    if (dot) mk_rows<T, K, true><<<grid, kBlock, 0, s>>>(n, rp, ci, av, g, e, partials, pmask);
    else mk_rows<T, K, false><<<grid, kBlock, 0, s>>>(n, rp, ci, av, g, e, partials, pmask);
    HIPC(hipGetLastError());
}

template <class T>
const T *vvals(const Csr &A);
template <>
const double *vvals<double>(const Csr &A) { return A.v; }
template <>
const float *vvals<float>(const Csr &A) { return A.v32; }
template <class T>
const T *vwd(const Level &L);
template <>
const double *vwd<double>(const Level &L) { return L.wd; }
template <>
const float *vwd<float>(const Level &L) { return L.wd32; }
template <class T>
const T *vawd(const Level &L);
template <>
const double *vawd<double>(const Level &L) { return L.awd; }
template <>
const float *vawd<float>(const Level &L) { return L.awd32; }

// One V-cycle on the K-column block R -> Z (level-0 post-smoothing writes
// the per-column r.z partials when dot).
template <class T, int K>
void mvcycle(Engine &E, bool dot, hipStream_t s) {
    Hier &h = *E.h;
    const int L = h.nlev - 1;
    if (L == 0) {  // one level: direct solve, then the r.z partials
        mk_coarse<double, K><<<(h.nL + kBlock / K - 1) / (kBlock / K), kBlock, 0, s>>>(h.nL, h.cinv, E.R, E.Z);
        if (dot) mk_dot<K><<<E.nb_vec, kBlock, 0, s>>>(E.n, E.R, E.Z, E.prz);
        HIPC(hipGetLastError());
        return;
    }
    auto Tp = [](void *p) { return static_cast<T *>(p); };
    T *sv[CAMG_MAX_LEVELS] = {};
    for (int l = 0; l < L; ++l) {
        Level &Lv = h.lev[l];
        Engine::Lv &B = E.lv[l];
        const int nl = Lv.A.nr;
        T *s0 = Tp(B.s), *t0 = Tp(B.t), *r0 = Tp(B.r);
        if (l == 0)
            launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vawd<T>(Lv), B.grid, s, MGather<T, K, double>{E.R},
                                   MEPre<T, K, double>{vwd<T>(Lv), E.R, s0, r0}, nullptr, false);
        else
            launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vawd<T>(Lv), B.grid, s, MGather<T, K>{Tp(B.y)},
                                   MEPre<T, K, T>{vwd<T>(Lv), Tp(B.y), s0, r0}, nullptr, false);
        for (int it = 1; it < h.prm.nu_pre; ++it) {
            if (l == 0)
                launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vvals<T>(Lv.A), B.grid, s, MGather<T, K>{s0},
                                       MEPost<T, K, double, T>{vwd<T>(Lv), E.R, s0, t0}, nullptr, false);
            else
                launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vvals<T>(Lv.A), B.grid, s, MGather<T, K>{s0},
                                       MEPost<T, K, T, T>{vwd<T>(Lv), Tp(B.y), s0, t0}, nullptr, false);
            std::swap(s0, t0);
        }
        if (h.prm.nu_pre > 1) {
            if (l == 0)
                launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vvals<T>(Lv.A), B.grid, s, MGather<T, K>{s0},
                                       MEResid<T, K, double>{E.R, r0}, nullptr, false);
            else
                launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vvals<T>(Lv.A), B.grid, s, MGather<T, K>{s0},
                                       MEResid<T, K, T>{Tp(B.y), r0}, nullptr, false);
        }
        sv[l] = s0;
        launch_mrows_any<T, K>(Lv.R.nr, Lv.R.rp, Lv.R.ci, vvals<T>(Lv.R), B.gridR, s, MGather<T, K>{r0},
                               MESpmv<T, K, false>{Tp(E.lv[l + 1].y)}, nullptr, false);
    }
    mk_coarse<T, K><<<(h.nL + kBlock / K - 1) / (kBlock / K), kBlock, 0, s>>>(h.nL, h.cinv, Tp(E.lv[L].y),
                                                                              Tp(E.lv[L].z));
    HIPC(hipGetLastError());
    for (int l = L - 1; l >= 0; --l) {
        Level &Lv = h.lev[l];
        Engine::Lv &B = E.lv[l];
        const int nl = Lv.A.nr;
        launch_mrows_any<T, K>(Lv.P.nr, Lv.P.rp, Lv.P.ci, vvals<T>(Lv.P), B.gridP, s, MGather<T, K>{Tp(E.lv[l + 1].z)},
                               MESpmv<T, K, true>{sv[l]}, nullptr, false);
        T *s0 = sv[l];
        T *t0 = (s0 == Tp(B.s)) ? Tp(B.t) : Tp(B.s);
        for (int it = 0; it + 1 < h.prm.nu_post; ++it) {
            if (l == 0)
                launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vvals<T>(Lv.A), B.grid, s, MGather<T, K>{s0},
                                       MEPost<T, K, double, T>{vwd<T>(Lv), E.R, s0, t0}, nullptr, false);
            else
                launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vvals<T>(Lv.A), B.grid, s, MGather<T, K>{s0},
                                       MEPost<T, K, T, T>{vwd<T>(Lv), Tp(B.y), s0, t0}, nullptr, false);
            std::swap(s0, t0);
        }
        if (l == 0)
            launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vvals<T>(Lv.A), B.grid, s, MGather<T, K>{s0},
                                   MEPost<T, K, double, double>{vwd<T>(Lv), E.R, s0, E.Z}, E.prz, dot);
        else
            launch_mrows_any<T, K>(nl, Lv.A.rp, Lv.A.ci, vvals<T>(Lv.A), B.grid, s, MGather<T, K>{s0},
                                   MEPost<T, K, T, T>{vwd<T>(Lv), Tp(B.y), s0, Tp(B.z)}, nullptr, false);
    }
}

template <int K>
void miteration(Engine &E, int par, hipStream_t s) {
    Hier &h = *E.h;
    const Csr &A = h.lev[0].A;
    mk_check<K><<<1, kRed, 0, s>>>(E.pr2, E.nb_vec, E.st, E.hist, E.cap, E.hflag_dev);
    HIPC(hipGetLastError());
    if (E.mixed) mvcycle<float, K>(E, true, s);
    else mvcycle<double, K>(E, true, s);
    // the r.z partials come from a kernel on the n_0 rows: lv[0].grid == nb_vec blocks
    mk_fin_rz<K><<<1, kRed, 0, s>>>(E.prz, E.nb_vec, E.st);
    const double *beta =
        reinterpret_cast<const double *>(reinterpret_cast<const char *>(E.st) + offsetof(MState, beta));
    launch_mrows_any<double, K>(A.nr, A.rp, A.ci, A.v, E.lv[0].grid, s, MGDir<K>{E.Z, E.P[par], beta},
                                MEDir<K>{E.Z, E.P[par], beta, E.P[1 - par], E.Q}, E.ppq, true);
    mk_fin_pq<K><<<1, kRed, 0, s>>>(E.ppq, E.lv[0].grid, E.st);
    mk_update<K><<<E.nb_vec, kBlock, 0, s>>>(E.n, E.P[1 - par], E.Q, E.X, E.R, E.pr2, E.st);
    HIPC(hipGetLastError());
}

#define CAMG_K_SWITCH(K, ...)                            \
    switch (K) {                                         \
    case 1: { constexpr int KK = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int KK = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int KK = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int KK = 32; __VA_ARGS__; } break; \
    default: { constexpr int KK = 64; __VA_ARGS__; } break; \
    }

void m_destroy_graphs(Engine &E) {
    for (int p = 0; p < 2; ++p) {
        if (E.gexec[p]) (void)hipGraphExecDestroy(E.gexec[p]);
        if (E.graph[p]) (void)hipGraphDestroy(E.graph[p]);
        E.gexec[p] = nullptr;
        E.graph[p] = nullptr;
    }
    E.graph_ok = false;
}

void m_build_graphs(Engine &E) {
    m_destroy_graphs(E);
    if (!E.cap_stream) HIPC(hipStreamCreateWithFlags(&E.cap_stream, hipStreamNonBlocking));
    for (int p = 0; p < 2; ++p) {
        HIPC(hipStreamBeginCapture(E.cap_stream, hipStreamCaptureModeThreadLocal));
        try {
            CAMG_K_SWITCH(E.K, miteration<KK>(E, p, E.cap_stream));
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(E.cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        HIPC(hipStreamEndCapture(E.cap_stream, &E.graph[p]));
        HIPC(hipGraphInstantiate(&E.gexec[p], E.graph[p], nullptr, nullptr, 0));
    }
    E.graph_ok = true;
}

void m_launch_iteration(Engine &E, hipStream_t s) {
    if (E.use_graph && !E.graph_ok) {
        try {
            m_build_graphs(E);
        } catch (const Error &) {
            m_destroy_graphs(E);
            E.use_graph = false;
        }
    }
    if (E.use_graph && E.graph_ok) HIPC(hipGraphLaunch(E.gexec[E.par], s));
    else CAMG_K_SWITCH(E.K, miteration<KK>(E, E.par, s));
    E.par ^= 1;
}

}  // namespace

Engine::~Engine() {
    m_destroy_graphs(*this);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hflag) (void)hipHostFree(hflag);
}

int64_t engine_footprint(const Hier &h, int K) {
    const int64_t n = h.lev[0].A.nr;
    const bool mixed = h.prm.precision == CAMG_MIXED_FP32;
    int64_t b = 7 * n * K * 8;  // X, R, B, Z, P0, P1, Q
    for (int l = 0; l < h.nlev; ++l) b += 5 * (int64_t)h.lev[l].A.nr * K * (mixed ? 4 : 8);
    b += 4 * (int64_t)kMGridMax * K * 8 + sizeof(MState);
    return b;
}

Engine *engine_create(Hier &h, int K, int cap, hipStream_t s) {
    if (K < 1 || K > kMaxSlots || (K & (K - 1))) fail(CAMG_E_ARG, "slot count must be a power of two in [1, 64]");
    std::unique_ptr<Engine> E(new Engine());
    E->h = &h;
    E->K = K;
    E->n = h.lev[0].A.nr;
    E->mixed = h.prm.precision == CAMG_MIXED_FP32;
    E->stream = s;
    const size_t blk = (size_t)E->n * K;
    E->X = E->pool.alloc<double>(blk);
    E->R = E->pool.alloc<double>(blk);
    E->Bk = E->pool.alloc<double>(blk);
    E->Z = E->pool.alloc<double>(blk);
    E->P[0] = E->pool.alloc<double>(blk);
    E->P[1] = E->pool.alloc<double>(blk);
    E->Q = E->pool.alloc<double>(blk);
    const size_t vb = E->mixed ? 4 : 8;
    E->lv.resize(h.nlev);
    for (int l = 0; l < h.nlev; ++l) {
        const Level &L = h.lev[l];
        Engine::Lv &B = E->lv[l];
        const size_t nb = (size_t)L.A.nr * K * vb;
        if (l > 0) {
            B.y = E->pool.raw(nb);
            B.z = E->pool.raw(nb);
        }
        B.s = E->pool.raw(nb);
        B.t = E->pool.raw(nb);
        B.r = E->pool.raw(nb);
        B.grid = mgrid(L.A.nr, K);
        if (l < h.nlev - 1) {
            B.gridP = mgrid(L.P.nr, K);
            B.gridR = mgrid(L.R.nr, K);
        }
    }
    E->nb_vec = mgrid(E->n, K);
    E->pr2 = E->pool.alloc<double>((size_t)kMGridMax * K);
    E->prz = E->pool.alloc<double>((size_t)kMGridMax * K);
    E->ppq = E->pool.alloc<double>((size_t)kMGridMax * K);
    E->ptmp = E->pool.alloc<double>((size_t)kMGridMax * K);
    E->sc = E->pool.alloc<double>(kMaxSlots);
    E->st = E->pool.alloc<MState>(1);
    E->cap = cap;
    E->hist = E->pool.alloc<double>((size_t)K * std::max(cap, 1));
    // the PCG blocks start zeroed and every slot inactive (unused columns
    // are computed along but never read; their values never mix with others)
    HIPC(hipMemsetAsync(E->st, 0, sizeof(MState), s));
    for (double *p : {E->X, E->R, E->Bk, E->Z, E->P[0], E->P[1], E->Q}) HIPC(hipMemsetAsync(p, 0, blk * 8, s));
    for (auto &B : E->lv)
        for (void *p : {B.y, B.s, B.t, B.r, B.z})
            if (p) HIPC(hipMemsetAsync(p, 0, (size_t)h.lev[&B - &E->lv[0]].A.nr * K * vb, s));
    HIPC(hipMemsetAsync(E->pr2, 0, (size_t)kMGridMax * K * 8, s));
    HIPC(hipHostMalloc((void **)&E->hflag, 4 * sizeof(int32_t), hipHostMallocMapped));
    HIPC(hipHostGetDevicePointer((void **)&E->hflag_dev, E->hflag, 0));
    E->hflag[0] = 0;
    HIPC(hipStreamSynchronize(s));
    return E.release();
}

void engine_start_slots(Engine &E, const SlotMap &q, const double *B, int ldb, double rtol, int max_iter,
                        hipStream_t s) {
    CAMG_K_SWITCH(E.K, (mk_start<KK><<<E.nb_vec, kBlock, 0, s>>>(E.n, q, B, ldb, E.X, E.R, E.Bk, E.P[0], E.P[1], rtol,
                                                                  max_iter, E.pr2, E.st)));
    HIPC(hipGetLastError());
    E.hflag[0] = 1;
}

void engine_start(Engine &E, int c0, int m, const double *B, int ldb, double rtol, int max_iter, hipStream_t s) {
    if (c0 < 0 || m < 1 || c0 + m > E.K) fail(CAMG_E_ARG, "slot range out of bounds");
    SlotMap q;
    for (int c = 0; c < kMaxSlots; ++c) q.q[c] = (c >= c0 && c < c0 + m) ? (int8_t)(c - c0) : (int8_t)-1;
    engine_start_slots(E, q, B, ldb, rtol, max_iter, s);
}

// Enqueue `iters` iterations and a stopping test; no wait.
void engine_launch(Engine &E, int iters, hipStream_t s) {
    for (int k = 0; k < iters; ++k) m_launch_iteration(E, s);
    CAMG_K_SWITCH(E.K, (mk_check<KK><<<1, kRed, 0, s>>>(E.pr2, E.nb_vec, E.st, E.hist, E.cap, E.hflag_dev)));
    HIPC(hipGetLastError());
}

// Enqueue the per-column snapshot into the device buffer `snap` (with the
// true residual sums when true_res); no wait.
void engine_snapshot(Engine &E, bool true_res, EngineSnap *snap, hipStream_t s) {
    if (true_res) {
        const Csr &A = E.h->lev[0].A;
        CAMG_K_SWITCH(E.K, (launch_mrows_any<double, KK>(A.nr, A.rp, A.ci, A.v, E.lv[0].grid, s,
                                                           MGather<double, KK>{E.X}, MERes<KK>{E.Bk, nullptr, 0ull},
                                                           E.ptmp, true)));
        CAMG_K_SWITCH(E.K, (mk_sum<KK><<<1, kRed, 0, s>>>(E.ptmp, E.lv[0].grid, E.sc)));
    }
    CAMG_K_SWITCH(E.K, (mk_snap<KK><<<1, 64, 0, s>>>(E.st, true_res ? E.sc : nullptr, snap)));
    HIPC(hipGetLastError());
}

void engine_release_mask(Engine &E, unsigned long long mask, hipStream_t s) {
    if (!mask) return;
    CAMG_K_SWITCH(E.K, (mk_release<KK><<<1, 64, 0, s>>>(E.st, mask)));
    HIPC(hipGetLastError());
}

void engine_gather_x(Engine &E, const SlotMap &q, int k, double *out, hipStream_t s) {
    const int64_t tot = (int64_t)E.n * k;
    const int grid = (int)std::min<int64_t>((tot + kBlock - 1) / kBlock, 4096);
    CAMG_K_SWITCH(E.K, (mk_gather_cols<KK><<<std::max(grid, 1), kBlock, 0, s>>>(E.n, k, q, E.X, out)));
    HIPC(hipGetLastError());
}

int engine_n(const Engine &E) { return E.n; }

// Run up to `iters` iterations (or until no column is running); polls one
// iteration behind.  Returns the number of running columns at the end.
int engine_step(Engine &E, int iters, hipStream_t s) {
    hipEvent_t ev[2];
    HIPC(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    HIPC(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
    } eg{ev};
    volatile int32_t *flag = E.hflag;
    for (int k = 0; k < iters; ++k) {
        m_launch_iteration(E, s);
        HIPC(hipEventRecord(ev[k & 1], s));
        if (k >= 1) {
            HIPC(hipEventSynchronize(ev[(k - 1) & 1]));
            if (flag[0] == 0) break;
        }
    }
    // stopping test for the residuals just formed
    CAMG_K_SWITCH(E.K, (mk_check<KK><<<1, kRed, 0, s>>>(E.pr2, E.nb_vec, E.st, E.hist, E.cap, E.hflag_dev)));
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));
    return flag[0];
}

void engine_slot_state(Engine &E, int32_t *iters, int32_t *done, int32_t *status, hipStream_t s) {
    MState st;
    HIPC(hipMemcpyAsync(&st, E.st, sizeof(MState), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int c = 0; c < E.K; ++c) {
        if (iters) iters[c] = st.iter[c];
        if (done) done[c] = st.active[c] ? (st.done[c] ? 1 : 0) : -1;
        if (status) status[c] = st.status[c];
    }
}

// true ||b - A x|| / ||b|| of every slot (host array of K)
void engine_true_res(Engine &E, double *rel, hipStream_t s) {
    const Csr &A = E.h->lev[0].A;
    CAMG_K_SWITCH(E.K, (launch_mrows_any<double, KK>(A.nr, A.rp, A.ci, A.v, E.lv[0].grid, s, MGather<double, KK>{E.X},
                                                       MERes<KK>{E.Bk, nullptr, 0ull}, E.ptmp, true)));
    double *part = E.ptmp;
    CAMG_K_SWITCH(E.K, (mk_sum<KK><<<1, kRed, 0, s>>>(part, E.lv[0].grid, E.sc)));
    HIPC(hipGetLastError());
    double t2[kMaxSlots];
    MState st;
    HIPC(hipMemcpyAsync(t2, E.sc, sizeof(double) * E.K, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(&st, E.st, sizeof(MState), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int c = 0; c < E.K; ++c) rel[c] = st.bnorm[c] > 0.0 ? std::sqrt(t2[c]) / st.bnorm[c] : 0.0;
}

// copy columns [c0, c0+m) of X to the n-by-m block X (row stride ldx, device)
void engine_copy_x(Engine &E, int c0, int m, double *X, int ldx, hipStream_t s) {
    HIPC(hipMemcpy2DAsync(X, sizeof(double) * ldx, E.X + c0, sizeof(double) * E.K, sizeof(double) * m, E.n,
                          hipMemcpyDeviceToDevice, s));
}

// mark columns [c0, c0+m) free
void engine_release(Engine &E, int c0, int m, hipStream_t s) {
    unsigned long long mask = 0;
    for (int c = c0; c < c0 + m; ++c) mask |= 1ull << c;
    engine_release_mask(E, mask, s);
    HIPC(hipStreamSynchronize(s));
}

void engine_hist(Engine &E, int c, double *host, int cap_out, int count, hipStream_t s) {
    const int m = std::min({cap_out, count, E.cap});
    if (m <= 0) return;
    HIPC(hipMemcpyAsync(host, E.hist + (size_t)c * E.cap, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
}

int engine_slots(const Engine &E) { return E.K; }

void engine_destroy(Engine *e) { delete e; }

// Mixed precision: restart the columns of `mask` from R = B - A X (their
// ||r||^2 partials are replaced too; the other columns are untouched).
void engine_replace(Engine &E, unsigned long long mask, hipStream_t s) {
    if (!mask) return;
    const Csr &A = E.h->lev[0].A;
    CAMG_K_SWITCH(E.K, (launch_mrows_any<double, KK>(A.nr, A.rp, A.ci, A.v, E.lv[0].grid, s, MGather<double, KK>{E.X},
                                                       MERes<KK>{E.Bk, E.R, mask}, E.pr2, true, mask)));
    CAMG_K_SWITCH(E.K, (mk_restart<KK><<<1, 64, 0, s>>>(E.st, mask)));
    HIPC(hipGetLastError());
    E.hflag[0] = 1;
}

}  // namespace camg
