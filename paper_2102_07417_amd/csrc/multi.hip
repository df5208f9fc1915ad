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
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include <hip/hip_ext.h>

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
// A lane owns V consecutive columns of its row (V * sizeof(T) = 16 bytes
// where K allows), so a gather of row j is one 16-byte load per lane and
// LPR = K / V lanes cover the row.
template <class T, int K>
struct Lay {
    static constexpr int V = (K * (int)sizeof(T) >= 16) ? 16 / (int)sizeof(T) : K;
    static constexpr int LPR = K / V;
    static constexpr int RPP = kBlock / LPR;  // rows per pass of a block
};

// V consecutive elements (16, 8 or 4k bytes, aligned to their size)
template <class X, int V>
__device__ __forceinline__ void vload(const X *p, X (&o)[V]) {
    constexpr int B = V * (int)sizeof(X);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int w = 0; w < B / 16; ++w) {
            const uint4 u = reinterpret_cast<const uint4 *>(p)[w];
            __builtin_memcpy(reinterpret_cast<char *>(o) + 16 * w, &u, 16);
        }
    } else if constexpr (B == 8) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        __builtin_memcpy(o, &u, 8);
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = p[v];
    }
}
template <class X, int V>
__device__ __forceinline__ void vstore(X *p, const X (&o)[V]) {
    constexpr int B = V * (int)sizeof(X);
    if constexpr (B % 16 == 0) {
#pragma unroll
        for (int w = 0; w < B / 16; ++w) {
            uint4 u;
            __builtin_memcpy(&u, reinterpret_cast<const char *>(o) + 16 * w, 16);
            reinterpret_cast<uint4 *>(p)[w] = u;
        }
    } else if constexpr (B == 8) {
        uint2 u;
        __builtin_memcpy(&u, o, 8);
        *reinterpret_cast<uint2 *>(p) = u;
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) p[v] = o[v];
    }
}

// Per-column sums over the block of the V accumulators of each lane:
// partials[blockIdx.x * K + c], lanes of the same column added in group order.
template <int K, int V>
__device__ __forceinline__ void block_col_sum_v(const double (&d)[V], double *partials, unsigned long long mask) {
    __shared__ double sh[kBlock * V];
#pragma unroll
    for (int v = 0; v < V; ++v) sh[threadIdx.x * V + v] = d[v];
    __syncthreads();
    constexpr int G = kBlock * V / K;
    if (threadIdx.x < K && ((mask >> threadIdx.x) & 1ull)) {
        double t = 0.0;
        for (int g = 0; g < G; ++g) t += sh[g * K + threadIdx.x];
        partials[(size_t)blockIdx.x * K + threadIdx.x] = t;
    }
    __syncthreads();
}

constexpr int kStage = 1024;  // CSR entries staged in LDS per chunk
constexpr int64_t kSweepL2 = (int64_t)3 << 19;  // bytes of gathered block rows a stripe sweep may keep in an XCD's L2
constexpr int kChunkRowsMax = 512;

// One row: acc(c0 .. c0+V) = sum_j a_ij g(j, .).  Entries U at a time,
// clamped to the row so all loads and gathers are unconditional and in
// flight together; products added in CSR order, padding skipped.
template <class T, int V, int U, class CI, class AV, class G>
__device__ __forceinline__ void row_acc(int e0, int e1, const CI *ci, const AV *av, const G &g, int c0, T (&acc)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = T(0);
    for (int eb = e0; eb < e1; eb += U) {
        int j[U];
        T a[U];
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int e = min(eb + t, e1 - 1);
            j[t] = ci[e];
            a[t] = av[e];
        }
        T x[U][V];
#pragma unroll
        for (int t = 0; t < U; ++t) g.template get<V>(j[t], c0, x[t]);
#pragma unroll
        for (int t = 0; t < U; ++t)
            if (eb + t < e1) {
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] += a[t] * x[t][v];
            }
    }
}

// out(i, .) = sum_j a_ij g(j, .); epi(i, c0, acc, dot).  The rows are cut
// into chunks of `crows` rows; each XCD takes a contiguous eighth of the
// chunks and its blocks sweep it together, block j taking chunks j, j + B,
// ... (B blocks per XCD), so the chunks in flight on an XCD are neighbours
// and the rows they gather (a stencil's nearby rows) are shared through its
// L2 instead of being fetched again from the memory-side cache.  With
// `stage`, a chunk whose entries fit is first copied to LDS (indices,
// values, row pointers, coalesced) and the group's lanes read the entries
// there; otherwise they read them from memory.
//
// With pc > 0 the XCD's chunks are taken in stripes: its slab is read as
// planes of pc chunks (pc chunks ~ the distance from a row to its farthest
// neighbour, e.g. one plane of a 3D grid), each cut into stripes of wc
// chunks, and the sweep goes stripe by stripe, plane by plane within a
// stripe.  The block rows a chunk gathers from the planes before and after
// it are then gathered again while they are still in the XCD's L2, instead
// of a whole plane later (a plane of block rows exceeds the L2).  Every
// chunk is taken once; only the order, and so which block adds a row's dot
// terms, changes.
template <class T, int K, bool DOT, int U, class G, class E>
__global__ void __launch_bounds__(kBlock) mk_rows(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                  const T *__restrict__ av, G g, E epi, double *partials,
                                                  unsigned long long pmask, int crows, int stage, int pc, int wc) {
    using L = Lay<T, K>;
    constexpr int V = L::V, LPR = L::LPR, RPP = L::RPP;
    __shared__ int32_t s_ci[kStage];
    __shared__ T s_av[kStage];
    __shared__ int32_t s_rp[kChunkRowsMax + 1];
    const int lane = threadIdx.x % LPR, grp = threadIdx.x / LPR;
    const int c0 = lane * V;
    g.prep(c0);
    epi.prep(c0);
    const int nch = (n + crows - 1) / crows;
    const int xcd = blockIdx.x & 7, bx = gridDim.x >> 3, jb = blockIdx.x >> 3;
    const int ch0 = (int)((int64_t)xcd * nch / 8), ch1 = (int)((int64_t)(xcd + 1) * nch / 8);
    double dot[V];
#pragma unroll
    for (int v = 0; v < V; ++v) dot[v] = 0.0;
    const int m = ch1 - ch0;
    const bool striped = pc > 0 && wc < pc;
    const int zpl = striped ? (m + pc - 1) / pc : 1;  // planes of the slab
    const int nst = striped ? (pc + wc - 1) / wc : 1;   // stripes of a plane
    const int nq = striped ? nst * zpl * wc : m;
    for (int q = jb; q < nq; q += bx) {
        int ch = ch0 + q;
        if (striped) {  // q -> (stripe, plane, offset in the stripe)
            const int st = q / (zpl * wc), r = q - st * (zpl * wc);
            const int z = r / wc, off = st * wc + (r - z * wc);
            if (off >= pc || z * pc + off >= m) continue;
            ch = ch0 + z * pc + off;
        }
        const int a = ch * crows, b = min(a + crows, n);
        const int E0 = rp[a], E1 = rp[b];
        if (stage && E1 - E0 <= kStage && b - a <= kChunkRowsMax) {
            __syncthreads();  // the previous chunk is done with the stage
            for (int t = threadIdx.x; t < E1 - E0; t += kBlock) {
                s_ci[t] = ci[E0 + t];
                s_av[t] = av[E0 + t];
            }
            for (int t = threadIdx.x; t <= b - a; t += kBlock) s_rp[t] = rp[a + t] - E0;
            __syncthreads();
            for (int i = a + grp; i < b; i += RPP) {
                typename E::template Pre<V> pre;
                epi.template load<V>(i, c0, pre);
                T acc[V];
                row_acc<T, V, U>(s_rp[i - a], s_rp[i - a + 1], s_ci, s_av, g, c0, acc);
                epi.template fin<V>(i, c0, acc, pre, dot);
            }
        } else {
            for (int i = a + grp; i < b; i += RPP) {
                typename E::template Pre<V> pre;
                epi.template load<V>(i, c0, pre);
                T acc[V];
                row_acc<T, V, U>(rp[i], rp[i + 1], ci, av, g, c0, acc);
                epi.template fin<V>(i, c0, acc, pre, dot);
            }
        }
    }
    if constexpr (DOT) block_col_sum_v<K, V>(dot, partials, pmask);
}

// rows per chunk of a matrix with `nnz` entries in `nr` rows
template <class T, int K>
int chunk_rows(int64_t nr, int64_t nnz) {
    constexpr int RPP = Lay<T, K>::RPP;
    const double mean = nr > 0 ? std::max(1.0, (double)nnz / (double)nr) : 1.0;
    int r = (int)(0.75 * kStage / mean) / RPP * RPP;
    r = std::min(r, kChunkRowsMax / RPP * RPP);
    return std::max(r, RPP);
}

template <class T, int K, class TX = T>
struct MGather {
    static constexpr int kU = 8;
    static constexpr int kRowBytes = K * (int)sizeof(TX);  // bytes of one gathered block row
    __device__ void prep(int) {}
    const TX *x;
    template <int V>
    __device__ void get(int j, int c0, T (&o)[V]) const {
        TX u[V];
        vload<TX, V>(x + (size_t)j * K + c0, u);
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = (T)u[v];
    }
};

// Epilogues: load(i, c0, pre) issues the row's epilogue reads, which the
// row loop calls before the row's gathers so that both wait together;
// fin(i, c0, acc, pre, dot) completes the row.
template <class T, int K, class TY>
struct MEPre {  // S = wd Y, R = Y - (A wd) Y  (values pre-scaled by wd)
    __device__ void prep(int) {}
    const T *wd;
    const TY *y;
    T *s, *r;
    template <int V>
    struct Pre {
        TY y[V];
        T w;
    };
    template <int V>
    __device__ void load(int i, int c0, Pre<V> &p) const {
        vload<TY, V>(y + (size_t)i * K + c0, p.y);
        p.w = wd[i];
    }
    template <int V>
    __device__ void fin(int i, int c0, const T (&acc)[V], const Pre<V> &p, double (&)[V]) const {
        const size_t o = (size_t)i * K + c0;
        T sv[V], rv[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T yi = (T)p.y[v];
            sv[v] = p.w * yi;
            rv[v] = yi - acc[v];
        }
        vstore<T, V>(s + o, sv);
        vstore<T, V>(r + o, rv);
    }
};
template <class T, int K, class TY, class TZ>
struct MEPost {  // Z = S + wd (Y - A S); dot += Y Z
    __device__ void prep(int) {}
    const T *wd;
    const TY *y;
    const T *s;
    TZ *z;
    template <int V>
    struct Pre {
        TY y[V];
        T s[V];
        T w;
    };
    template <int V>
    __device__ void load(int i, int c0, Pre<V> &p) const {
        const size_t o = (size_t)i * K + c0;
        vload<TY, V>(y + o, p.y);
        vload<T, V>(s + o, p.s);
        p.w = wd[i];
    }
    template <int V>
    __device__ void fin(int i, int c0, const T (&acc)[V], const Pre<V> &p, double (&dot)[V]) const {
        const size_t o = (size_t)i * K + c0;
        TZ zv[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const T zi = p.s[v] + p.w * ((T)p.y[v] - acc[v]);
            zv[v] = (TZ)zi;
            dot[v] += (double)p.y[v] * (double)zv[v];
        }
        vstore<TZ, V>(z + o, zv);
    }
};
template <class T, int K, class TY>
struct MEResid {
    __device__ void prep(int) {}
    const TY *y;
    T *r;
    template <int V>
    struct Pre {
        TY y[V];
    };
    template <int V>
    __device__ void load(int i, int c0, Pre<V> &p) const {
        vload<TY, V>(y + (size_t)i * K + c0, p.y);
    }
    template <int V>
    __device__ void fin(int i, int c0, const T (&acc)[V], const Pre<V> &p, double (&)[V]) const {
        T rv[V];
#pragma unroll
        for (int v = 0; v < V; ++v) rv[v] = (T)p.y[v] - acc[v];
        vstore<T, V>(r + (size_t)i * K + c0, rv);
    }
};
template <class T, int K, bool ADD>
struct MESpmv {
    __device__ void prep(int) {}
    T *out;
    template <int V>
    struct Pre {
        T o[V];
    };
    template <int V>
    __device__ void load(int i, int c0, Pre<V> &p) const {
        if (ADD) vload<T, V>(out + (size_t)i * K + c0, p.o);
    }
    template <int V>
    __device__ void fin(int i, int c0, const T (&acc)[V], const Pre<V> &p, double (&)[V]) const {
        T ov[V];
#pragma unroll
        for (int v = 0; v < V; ++v) ov[v] = ADD ? p.o[v] + acc[v] : acc[v];
        vstore<T, V>(out + (size_t)i * K + c0, ov);
    }
};
template <int K>
struct MEPQ {  // Q = A P; dot += P.Q (own row of P read back)
    __device__ void prep(int) {}
    const double *p;
    double *q;
    template <int V>
    struct Pre {
        double p[V];
    };
    template <int V>
    __device__ void load(int i, int c0, Pre<V> &pr) const {
        vload<double, V>(p + (size_t)i * K + c0, pr.p);
    }
    template <int V>
    __device__ void fin(int i, int c0, const double (&acc)[V], const Pre<V> &pr, double (&dot)[V]) const {
#pragma unroll
        for (int v = 0; v < V; ++v) dot[v] += pr.p[v] * acc[v];
        vstore<double, V>(q + (size_t)i * K + c0, acc);
    }
};
template <int K>
struct MERes {  // d = B - A X; dot += d^2; R = d for the columns of `mask`
    __device__ void prep(int) {}
    const double *b;
    double *out;
    float *out32;  // FP32 copy of R (mixed precision) or null
    unsigned long long mask;
    template <int V>
    struct Pre {
        double b[V];
    };
    template <int V>
    __device__ void load(int i, int c0, Pre<V> &p) const {
        vload<double, V>(b + (size_t)i * K + c0, p.b);
    }
    template <int V>
    __device__ void fin(int i, int c0, const double (&acc)[V], const Pre<V> &p, double (&dot)[V]) const {
        const size_t o = (size_t)i * K + c0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const double d = p.b[v] - acc[v];
            if (out && ((mask >> (c0 + v)) & 1ull)) {
                out[o + v] = d;
                if (out32) out32[o + v] = (float)d;
            }
            dot[v] += d * d;
        }
    }
};

// ------------------------------------------------------------------ elementwise / state kernels
// Start the columns c with q.q[c] >= 0 from column q.q[c] of B (n-by-m
// row-major, row stride ldb): X = 0, R = B, both P = 0; state reset;
// partials of ||b||^2 for them.
template <int K>
__global__ void __launch_bounds__(kBlock) mk_start(int n, SlotMap q, const double *__restrict__ B, int ldb,
                                                   double *X, double *R, float *R32, double *B0, double *P0, double *P1,
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
            if (R32) R32[o] = (float)bi;
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

// largest |j - i| over the entries of a square CSR matrix with sorted rows
// (first and last column of every row), as an unsigned maximum into *out
__global__ void __launch_bounds__(kBlock) mk_band(int n, const int32_t *rp, const int32_t *ci,
                                                  unsigned long long *out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    int b = 0;
    if (i < n && rp[i + 1] > rp[i]) b = max(i - ci[rp[i]], ci[rp[i + 1] - 1] - i);
    const unsigned long long m = block_max_u64<kBlock>((unsigned long long)b);
    if (threadIdx.x == 0) atomicMax(out, m);
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
                                                    double *X, double *R, float *R32, double *pr2,
                                                    const MState *st) {
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
            if (R32) R32[o] = (float)ri;
        }
        acc += ri * ri;
    }
    block_col_sum<K>(acc, pr2);
}

// P_new = Z + beta_c P_old for every column (beta_c = 0 for columns that
// are not running, which leaves P_new = Z: finite and never used)
template <int K, class TZ>
__global__ void __launch_bounds__(kBlock) mk_pnew(int n, const TZ *__restrict__ Z, const double *__restrict__ Pold,
                                                  double *__restrict__ Pnew, const MState *st) {
    const int64_t tot = (int64_t)n * K;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < tot; t += (int64_t)gridDim.x * kBlock) {
        const int c = (int)(t % K);
        Pnew[t] = (double)Z[t] + st->beta[c] * Pold[t];
    }
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

// last level: Z = Ainv Y for a K-column block, a dense FP64 product on the
// matrix cores.  One wavefront per 16x16 tile of Z runs
// v_mfma_f64_16x16x4f64 over the inner dimension in steps of 4: lane l holds
// A(i0 + l%16, k0 + l/16) and Y(k0 + l/16, j0 + l%16), and its four results
// r = 0..3 are rows i0 + l/16 + 4r of column j0 + l%16 (the layout measured
// on gfx950).  Out-of-range rows, columns
// and inner indices contribute zeros.  Column j of Z depends only on column
// j of Y.
typedef double mk_d4 __attribute__((ext_vector_type(4)));
template <class T, int K>
__global__ void __launch_bounds__(kBlock) mk_coarse(int n, const double *__restrict__ cinv, const T *__restrict__ y,
                                                    T *__restrict__ z) {
    constexpr int TJ = (K + 15) / 16;  // column tiles
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int tile = blockIdx.x * (kBlock / 64) + wave;
    const int i0 = (tile / TJ) * 16, j0 = (tile % TJ) * 16;
    if (i0 >= n) return;  // uniform over the wavefront
    const int li = lane % 16, lk = lane / 16;
    const int ia = i0 + li, jb = j0 + li;
    const double *arow = cinv + (size_t)min(ia, n - 1) * n;
    mk_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < n; k0 += 4) {
        const int k = k0 + lk;
        const double a = (ia < n && k < n) ? arow[k] : 0.0;
        const double bv = (k < n && jb < K) ? (double)y[(size_t)k * K + jb] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + lk + 4 * r;
        if (i < n && jb < K) z[(size_t)i * K + jb] = (T)acc[r];
    }
}

template <class T, int K>
void launch_coarse(int n, const double *cinv, const T *y, T *z, hipStream_t s) {
    const int tiles = ((n + 15) / 16) * ((K + 15) / 16);
    mk_coarse<T, K><<<(tiles + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, s>>>(n, cinv, y, z);
    HIPC(hipGetLastError());
}

int mgrid(int n, int K) {
    const int rpp = kBlock / K;
    int g = (n + rpp - 1) / rpp;
    g = std::min(g, kMGridMax);
    return std::max(8, (g + 7) / 8 * 8);
}

}  // namespace

// ======================================================================= engine
// Schedule of the block-row kernels on one matrix: entries per unrolled
// step (0: the kernel's default), rows per chunk (0: from the mean row
// length), grid of the kernels without partial sums (0: the occupancy
// rule), whether chunks are staged in LDS.  Every schedule gives bitwise the
// same results: rows and products are added in the same order, and the
// grid (row partition) of a kernel producing partial sums never changes.
struct RowSched {
    int u = 0;
    int crows = 0;
    int grid = 0;
    int stage = 1;
    int band = 0;  // largest |j - i| of the matrix (square matrices; 0: plain sweep)
};

struct Engine {
    Hier *h = nullptr;
    int K = 0;
    int n = 0;
    bool mixed = false;
    Pool pool;
    double *X = nullptr, *R = nullptr, *Bk = nullptr, *P[2] = {nullptr, nullptr}, *Q = nullptr;
    void *Zv = nullptr;    // preconditioned residual: FP32 when the V-cycle is (it holds FP32 values), else FP64
    bool z32 = false;
    float *R32 = nullptr;  // FP32 copy of R kept by the PCG kernels (mixed precision)
    struct Lv {
        void *y = nullptr, *s = nullptr, *r = nullptr, *z = nullptr, *t = nullptr;
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
    int64_t iter_seq = 0;                       // iterations issued (strides of the kernel timing)
    hipEvent_t tev[2] = {nullptr, nullptr};     // a timed level-0 post-smoothing launch
    std::map<std::tuple<const void *, int, int>, RowSched> sched;  // (matrix, value bytes, kind)
    std::map<const void *, int> band;  // square matrices of the hierarchy: largest |j - i|
    int band_of(const Csr &M) const {
        auto it = band.find((const void *)&M);
        return it == band.end() ? 0 : it->second;
    }
    RowSched rs(const Csr &M, int vbytes, int kind) const {
        auto it = sched.find(std::make_tuple((const void *)&M, vbytes, kind));
        RowSched r = it == sched.end() ? RowSched{} : it->second;
        r.band = band_of(M);
        return r;
    }
    ~Engine();
};

namespace {

int device_cus() {
    static const int n = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                     hipSuccess)
            v = 256;
        return std::max(v, 8);
    }();
    return n;
}

// Grid of a block-row kernel on nr rows: one block per chunk, at most the
// blocks the device holds at once, a multiple of 8 (one share per XCD).
template <class T, int K, bool DOT, int U, class G, class Ep>
int rows_grid(int nr, int crows) {
    static const int occ = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, mk_rows<T, K, DOT, U, G, Ep>, kBlock, 0) != hipSuccess)
            b = 1;
        return std::max(b, 1);
    }();
    const int need = (nr + crows - 1) / crows;  // chunks
    const int cap = std::min(device_cus() * occ, kMGridMax) / 8 * 8;
    return std::max(8, std::min((need + 7) / 8 * 8, std::max(cap, 8)));
}

// events that the next block-row launch of this host thread records at its
// own start and end (armed by mrows_time_next, cleared by that launch)
thread_local hipEvent_t t_mev_start = nullptr, t_mev_stop = nullptr;
// events of the level-0 post-smoothing launch of the iteration being issued
// (set by a timed engine iteration, armed by the V-cycle right before it)
thread_local hipEvent_t t_mpost_start = nullptr, t_mpost_stop = nullptr;

void mrows_time_next(hipEvent_t a, hipEvent_t b) {
    t_mev_start = a;
    t_mev_stop = b;
}

template <class T, int K, bool DOT, int U, class G, class Ep>
int launch_mrows_u(const Csr &M, const T *av, hipStream_t s, const G &g, const Ep &e, double *partials,
                   unsigned long long pmask, int forced_grid, const RowSched &rs) {
    const int crows = rs.crows > 0 ? rs.crows : chunk_rows<T, K>(M.nr, M.nnz);
    int grid = forced_grid > 0 ? forced_grid : rows_grid<T, K, DOT, U, G, Ep>(M.nr, crows);
    if (!DOT && forced_grid <= 0 && rs.grid > 0) grid = rs.grid;
    // stripes when the block rows of a band (a plane of a grid) outgrow the
    // share of L2 they may take: five stripe-planes of gathered rows (the
    // planes before and after the ones in flight) fit kSweepL2
    int pc = 0, wc = 0;
    if (rs.band > 0) {
        const int64_t sw = std::max<int64_t>(crows, kSweepL2 / (5 * (int64_t)G::kRowBytes));  // rows per stripe
        if (sw < rs.band) {
            pc = (int)((rs.band + crows - 1) / crows);
            wc = (int)std::max<int64_t>(1, sw / crows);
        }
    }
    if (t_mev_start) {  // timed launch: the events bracket the kernel's execution
        hipEvent_t a = t_mev_start, b = t_mev_stop;
        t_mev_start = t_mev_stop = nullptr;
        hipExtLaunchKernelGGL(mk_rows<T, K, DOT, U, G, Ep>, dim3(grid), dim3(kBlock), 0, s, a, b, 0, M.nr, M.rp,
                              M.ci, av, g, e, partials, pmask, crows, rs.stage ? 1 : 0, pc, wc);
    } else {
        mk_rows<T, K, DOT, U><<<grid, kBlock, 0, s>>>(M.nr, M.rp, M.ci, av, g, e, partials, pmask, crows,
                                                      rs.stage ? 1 : 0, pc, wc);
    }
    HIPC(hipGetLastError());
    return grid;
}

// Launch on matrix M (values av) with schedule rs and return the grid used
// (forced_grid > 0: that grid, for partial sums that must line up with
// another kernel's; kernels with partial sums never take a tuned grid).
template <class T, int K, class G, class Ep>
int launch_mrows_any(const Csr &M, const T *av, hipStream_t s, const G &g, const Ep &e, double *partials, bool dot,
                     unsigned long long pmask = ~0ull, int forced_grid = 0, const RowSched &rs = RowSched{}) {
    const int u = rs.u ? rs.u : G::kU;
    if (dot) {
        if (u == 4) return launch_mrows_u<T, K, true, 4>(M, av, s, g, e, partials, pmask, forced_grid, rs);
        if (u == 7) return launch_mrows_u<T, K, true, 7>(M, av, s, g, e, partials, pmask, forced_grid, rs);
        return launch_mrows_u<T, K, true, 8>(M, av, s, g, e, partials, pmask, forced_grid, rs);
    }
    if (u == 4) return launch_mrows_u<T, K, false, 4>(M, av, s, g, e, partials, pmask, forced_grid, rs);
    if (u == 7) return launch_mrows_u<T, K, false, 7>(M, av, s, g, e, partials, pmask, forced_grid, rs);
    return launch_mrows_u<T, K, false, 8>(M, av, s, g, e, partials, pmask, forced_grid, rs);
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
int mvcycle(Engine &E, bool dot, hipStream_t s) {
    Hier &h = *E.h;
    const int L = h.nlev - 1;
    if (L == 0) {  // one level: direct solve, then the r.z partials
        double *Z = static_cast<double *>(E.Zv);  // one level: Z is FP64
        launch_coarse<double, K>(h.nL, h.cinv, E.R, Z, s);
        if (dot) mk_dot<K><<<E.nb_vec, kBlock, 0, s>>>(E.n, E.R, Z, E.prz);
        HIPC(hipGetLastError());
        return E.nb_vec;
    }
    auto Tp = [](void *p) { return static_cast<T *>(p); };
    T *sv[CAMG_MAX_LEVELS] = {};
    int g0 = 0;  // grid of the level-0 post-smoothing kernel (its r.z partials)
    for (int l = 0; l < L; ++l) {
        Level &Lv = h.lev[l];
        Engine::Lv &B = E.lv[l];
        T *s0 = Tp(B.s), *t0 = Tp(B.t), *r0 = Tp(B.r);
        if (l == 0) {
            if constexpr (sizeof(T) == 4)  // the FP32 copy of R holds exactly the values (T) R
                launch_mrows_any<T, K>(Lv.A, vawd<T>(Lv), s, MGather<T, K, float>{E.R32},
                                       MEPre<T, K, float>{vwd<T>(Lv), E.R32, s0, r0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
            else
                launch_mrows_any<T, K>(Lv.A, vawd<T>(Lv), s, MGather<T, K, double>{E.R},
                                       MEPre<T, K, double>{vwd<T>(Lv), E.R, s0, r0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
        }
        else
            launch_mrows_any<T, K>(Lv.A, vawd<T>(Lv), s, MGather<T, K>{Tp(B.y)},
                                   MEPre<T, K, T>{vwd<T>(Lv), Tp(B.y), s0, r0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
        for (int it = 1; it < h.prm.nu_pre; ++it) {
            if (l == 0)
                launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                       MEPost<T, K, double, T>{vwd<T>(Lv), E.R, s0, t0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
            else
                launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                       MEPost<T, K, T, T>{vwd<T>(Lv), Tp(B.y), s0, t0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
            std::swap(s0, t0);
        }
        if (h.prm.nu_pre > 1) {
            if (l == 0)
                launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                       MEResid<T, K, double>{E.R, r0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
            else
                launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                       MEResid<T, K, T>{Tp(B.y), r0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
        }
        sv[l] = s0;
        launch_mrows_any<T, K>(Lv.R, vvals<T>(Lv.R), s, MGather<T, K>{r0},
                               MESpmv<T, K, false>{Tp(E.lv[l + 1].y)}, nullptr, false, ~0ull, 0, E.rs(Lv.R, (int)sizeof(T), 0));
    }
    launch_coarse<T, K>(h.nL, h.cinv, Tp(E.lv[L].y), Tp(E.lv[L].z), s);
    for (int l = L - 1; l >= 0; --l) {
        Level &Lv = h.lev[l];
        Engine::Lv &B = E.lv[l];
        launch_mrows_any<T, K>(Lv.P, vvals<T>(Lv.P), s, MGather<T, K>{Tp(E.lv[l + 1].z)},
                               MESpmv<T, K, true>{sv[l]}, nullptr, false, ~0ull, 0, E.rs(Lv.P, (int)sizeof(T), 0));
        T *s0 = sv[l];
        T *t0 = (s0 == Tp(B.s)) ? Tp(B.t) : Tp(B.s);
        for (int it = 0; it + 1 < h.prm.nu_post; ++it) {
            if (l == 0)
                launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                       MEPost<T, K, double, T>{vwd<T>(Lv), E.R, s0, t0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
            else
                launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                       MEPost<T, K, T, T>{vwd<T>(Lv), Tp(B.y), s0, t0}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
            std::swap(s0, t0);
        }
        if (l == 0 && t_mpost_start) {  // a timed iteration: this launch records the events
            mrows_time_next(t_mpost_start, t_mpost_stop);
            t_mpost_start = t_mpost_stop = nullptr;
        }
        if (l == 0)
            g0 = E.z32 ? launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                                MEPost<T, K, double, float>{vwd<T>(Lv), E.R, s0,
                                                                            static_cast<float *>(E.Zv)},
                                                E.prz, dot, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0))
                       : launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                                MEPost<T, K, double, double>{vwd<T>(Lv), E.R, s0,
                                                                             static_cast<double *>(E.Zv)},
                                                E.prz, dot, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
        else
            launch_mrows_any<T, K>(Lv.A, vvals<T>(Lv.A), s, MGather<T, K>{s0},
                                   MEPost<T, K, T, T>{vwd<T>(Lv), Tp(B.y), s0, Tp(B.z)}, nullptr, false, ~0ull, 0, E.rs(Lv.A, (int)sizeof(T), 0));
    }
    return g0;
}

template <int K>
void miteration(Engine &E, int par, hipStream_t s) {
    Hier &h = *E.h;
    const Csr &A = h.lev[0].A;
    mk_check<K><<<1, kRed, 0, s>>>(E.pr2, E.nb_vec, E.st, E.hist, E.cap, E.hflag_dev);
    HIPC(hipGetLastError());
    const int nrz = E.mixed ? mvcycle<float, K>(E, true, s) : mvcycle<double, K>(E, true, s);
    mk_fin_rz<K><<<1, kRed, 0, s>>>(E.prz, nrz, E.st);
    if (E.z32)
        mk_pnew<K, float><<<E.nb_vec, kBlock, 0, s>>>(E.n, static_cast<const float *>(E.Zv), E.P[par], E.P[1 - par],
                                                      E.st);
    else
        mk_pnew<K, double><<<E.nb_vec, kBlock, 0, s>>>(E.n, static_cast<const double *>(E.Zv), E.P[par],
                                                       E.P[1 - par], E.st);
    const int npq = launch_mrows_any<double, K>(A, A.v, s, MGather<double, K>{E.P[1 - par]},
                                                MEPQ<K>{E.P[1 - par], E.Q}, E.ppq, true, ~0ull, 0, E.rs(A, 8, 1));
    mk_fin_pq<K><<<1, kRed, 0, s>>>(E.ppq, npq, E.st);
    mk_update<K><<<E.nb_vec, kBlock, 0, s>>>(E.n, E.P[1 - par], E.Q, E.X, E.R, E.R32, E.pr2, E.st);
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
    // kernel timing on the handle: every prof_stride-th iteration runs
    // without the graph, its level-0 post-smoothing launch bracketed by events
    Hier &h = *E.h;
    const bool timed = h.prof && (E.iter_seq % h.prof_stride) == h.prof_stride - 1 && E.h->nlev > 1;
    ++E.iter_seq;
    if (timed) {
        if (!E.tev[0]) {
            HIPC(hipEventCreate(&E.tev[0]));
            HIPC(hipEventCreate(&E.tev[1]));
        }
        t_mpost_start = E.tev[0];
        t_mpost_stop = E.tev[1];
        try {
            CAMG_K_SWITCH(E.K, miteration<KK>(E, E.par, s));
        } catch (...) {
            t_mpost_start = t_mpost_stop = nullptr;
            t_mev_start = t_mev_stop = nullptr;
            throw;
        }
        HIPC(hipEventSynchronize(E.tev[1]));
        float ms = 0.f;
        HIPC(hipEventElapsedTime(&ms, E.tev[0], E.tev[1]));
        h.prof_ms += ms;
        h.prof_launches += 1;
    } else if (E.use_graph && E.graph_ok) {
        HIPC(hipGraphLaunch(E.gexec[E.par], s));
    } else {
        CAMG_K_SWITCH(E.K, miteration<KK>(E, E.par, s));
    }
    E.par ^= 1;
}

// ------------------------------------------------------------------ autotuner
// Picks, per matrix of the hierarchy, the block-row schedule (entries per
// unrolled step, LDS chunk, grid) that runs fastest here, timing every
// candidate with HIP events when the engine is created; the choice is
// cached per matrix signature for the rest of the process.  Schedules never
// change results, so a tuned engine computes bitwise what an untuned one
// does.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int64_t, int, int, int>, RowSched> g_tune_cache;

template <class T, int K, class G, class Ep>
void tune_matrix(Engine &E, const Csr &M, const T *av, const G &g, const Ep &ep, double *partials, bool dot,
                 int kind, hipStream_t s) {
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, M.nr, M.nc, M.nnz, K, (int)sizeof(T), kind);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            E.sched[std::make_tuple((const void *)&M, (int)sizeof(T), kind)] = it->second;
            return;
        }
    }
    constexpr int RPP = Lay<T, K>::RPP;
    const int def = chunk_rows<T, K>(M.nr, M.nnz);
    RowSched plain{};
    plain.band = E.band_of(M);  // candidates sweep in the order the runs use
    const int rule = launch_mrows_any<T, K>(M, av, s, g, ep, partials, dot, ~0ull, 0, plain);  // warm; the rule grid
    std::vector<RowSched> cand;
    for (int u : {4, 7, 8})
        for (int cr : {def, std::max(RPP, def / 2 / RPP * RPP), RPP})
            for (int st : {1, 0})
                for (int gd : {0, std::max(8, rule / 2 / 8 * 8)}) {
                    if (gd != 0 && (dot || gd == rule)) continue;
                    if (!st && cr != def) continue;
                    cand.push_back(RowSched{u, cr, gd, st, plain.band});
                }
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } eg{e0, e1};
    RowSched best{};
    float best_ms = 1e30f;
    for (const RowSched &c : cand) {
        launch_mrows_any<T, K>(M, av, s, g, ep, partials, dot, ~0ull, 0, c);
        HIPC(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) launch_mrows_any<T, K>(M, av, s, g, ep, partials, dot, ~0ull, 0, c);
        HIPC(hipEventRecord(e1, s));
        HIPC(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPC(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    E.sched[std::make_tuple((const void *)&M, (int)sizeof(T), kind)] = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
}

template <class T, int K>
void autotune_t(Engine &E, hipStream_t s) {
    Hier &h = *E.h;
    const int L = h.nlev - 1;
    auto Tp = [](void *p) { return static_cast<T *>(p); };
    for (int l = 0; l < L; ++l) {
        const Level &Lv = h.lev[l];
        Engine::Lv &B = E.lv[l];
        tune_matrix<T, K>(E, Lv.A, vvals<T>(Lv.A), MGather<T, K>{Tp(B.s)}, MESpmv<T, K, false>{Tp(B.t)}, nullptr,
                          false, 0, s);
        tune_matrix<T, K>(E, Lv.R, vvals<T>(Lv.R), MGather<T, K>{Tp(B.r)}, MESpmv<T, K, false>{Tp(E.lv[l + 1].y)},
                          nullptr, false, 0, s);
        tune_matrix<T, K>(E, Lv.P, vvals<T>(Lv.P), MGather<T, K>{Tp(E.lv[l + 1].z)}, MESpmv<T, K, false>{Tp(B.t)},
                          nullptr, false, 0, s);
    }
    const Csr &A = h.lev[0].A;
    if (sizeof(T) != 8 || L == 0)
        tune_matrix<double, K>(E, A, A.v, MGather<double, K>{E.X}, MESpmv<double, K, false>{E.Q}, nullptr, false, 0,
                               s);
    // the product q = A p (with its p.q partials) takes the FP64 A_0 schedule; tune it with its own epilogue
    tune_matrix<double, K>(E, A, A.v, MGather<double, K>{E.P[0]}, MEPQ<K>{E.P[0], E.Q}, E.ptmp, true, 1, s);
}

void engine_autotune(Engine &E, hipStream_t s) {
    if (E.mixed) {
        CAMG_K_SWITCH(E.K, autotune_t<float, KK>(E, s));
    } else {
        CAMG_K_SWITCH(E.K, autotune_t<double, KK>(E, s));
    }
}

}  // namespace

Engine::~Engine() {
    m_destroy_graphs(*this);
    for (hipEvent_t e : tev)
        if (e) (void)hipEventDestroy(e);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hflag) (void)hipHostFree(hflag);
}

int64_t engine_footprint(const Hier &h, int K) {
    const int64_t n = h.lev[0].A.nr;
    const bool mixed = h.prm.precision == CAMG_MIXED_FP32;
    int64_t b = 7 * n * K * 8 + (mixed ? 4 * n * K : 0);  // X, R, B, Z, P0, P1, Q (+ FP32 R)
    for (int l = 0; l < h.nlev; ++l) b += 5 * (int64_t)h.lev[l].A.nr * K * (mixed ? 4 : 8);
    b += 4 * (int64_t)kMGridMax * K * 8 + sizeof(MState);
    return b;
}

Engine *engine_create(Hier &h, int K, int cap, hipStream_t s) {
    if (K < 1 || K > kMaxSlots || (K & (K - 1))) fail(CAMG_E_ARG, "slot count must be a power of two in [1, 64]");
    if (h.prm.smoother != CAMG_SMOOTH_JACOBI) fail(CAMG_E_ARG, "the multi-RHS engine runs the Jacobi smoother only");
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
    E->z32 = E->mixed && h.nlev > 1;
    E->Zv = E->pool.raw(blk * (E->z32 ? 4 : 8));
    E->P[0] = E->pool.alloc<double>(blk);
    E->P[1] = E->pool.alloc<double>(blk);
    E->Q = E->pool.alloc<double>(blk);
    if (E->mixed) E->R32 = E->pool.alloc<float>(blk);
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
    for (double *p : {E->X, E->R, E->Bk, E->P[0], E->P[1], E->Q}) HIPC(hipMemsetAsync(p, 0, blk * 8, s));
    HIPC(hipMemsetAsync(E->Zv, 0, blk * (E->z32 ? 4 : 8), s));
    if (E->R32) HIPC(hipMemsetAsync(E->R32, 0, blk * 4, s));
    for (auto &B : E->lv)
        for (void *p : {B.y, B.s, B.t, B.r, B.z})
            if (p) HIPC(hipMemsetAsync(p, 0, (size_t)h.lev[&B - &E->lv[0]].A.nr * K * vb, s));
    HIPC(hipMemsetAsync(E->pr2, 0, (size_t)kMGridMax * K * 8, s));
    HIPC(hipHostMalloc((void **)&E->hflag, 4 * sizeof(int32_t), hipHostMallocMapped));
    HIPC(hipHostGetDevicePointer((void **)&E->hflag_dev, E->hflag, 0));
    E->hflag[0] = 0;
    // the band of every level's matrix, for the stripe order of the block sweeps
    {
        unsigned long long *dband = E->pool.alloc<unsigned long long>(h.nlev);
        HIPC(hipMemsetAsync(dband, 0, sizeof(unsigned long long) * h.nlev, s));
        for (int l = 0; l < h.nlev; ++l) {
            const Csr &A = h.lev[l].A;
            if (A.nr > 0) mk_band<<<(A.nr + kBlock - 1) / kBlock, kBlock, 0, s>>>(A.nr, A.rp, A.ci, dband + l);
        }
        HIPC(hipGetLastError());
        std::vector<unsigned long long> hb(h.nlev);
        HIPC(hipMemcpyAsync(hb.data(), dband, sizeof(unsigned long long) * h.nlev, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        for (int l = 0; l < h.nlev; ++l) E->band[(const void *)&h.lev[l].A] = (int)hb[l];
    }
    if (h.autotune) engine_autotune(*E, s);
    HIPC(hipStreamSynchronize(s));
    return E.release();
}

void engine_start_slots(Engine &E, const SlotMap &q, const double *B, int ldb, double rtol, int max_iter,
                        hipStream_t s) {
    CAMG_K_SWITCH(E.K, (mk_start<KK><<<E.nb_vec, kBlock, 0, s>>>(E.n, q, B, ldb, E.X, E.R, E.R32, E.Bk, E.P[0], E.P[1], rtol,
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
        int nb = 0;
        CAMG_K_SWITCH(E.K, (nb = launch_mrows_any<double, KK>(A, A.v, s, MGather<double, KK>{E.X},
                                                                MERes<KK>{E.Bk, nullptr, nullptr, 0ull}, E.ptmp, true,
                                                                ~0ull, 0, E.rs(A, 8, 0))));
        CAMG_K_SWITCH(E.K, (mk_sum<KK><<<1, kRed, 0, s>>>(E.ptmp, nb, E.sc)));
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
    int nb = 0;
    CAMG_K_SWITCH(E.K, (nb = launch_mrows_any<double, KK>(A, A.v, s, MGather<double, KK>{E.X},
                                                            MERes<KK>{E.Bk, nullptr, nullptr, 0ull}, E.ptmp, true,
                                                            ~0ull, 0, E.rs(A, 8, 0))));
    CAMG_K_SWITCH(E.K, (mk_sum<KK><<<1, kRed, 0, s>>>(E.ptmp, nb, E.sc)));
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
    CAMG_K_SWITCH(E.K, (launch_mrows_any<double, KK>(A, A.v, s, MGather<double, KK>{E.X},
                                                       MERes<KK>{E.Bk, E.R, E.R32, mask}, E.pr2, true, mask, E.nb_vec,
                                                       E.rs(A, 8, 0))));
    CAMG_K_SWITCH(E.K, (mk_restart<KK><<<1, 64, 0, s>>>(E.st, mask)));
    HIPC(hipGetLastError());
    E.hflag[0] = 1;
}

}  // namespace camg
