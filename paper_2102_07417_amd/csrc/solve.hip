// Solve-phase kernels: the V-cycle of Alg. "AMG application in a V-cycle"
// with Jacobi smoothing (eq. smoother, M = D) and the PCG recurrence.
//
// Row kernels come in two shapes, chosen per matrix at set-up:
//  - tile: tile t holds the rows whose first nonzero lies in [t W, (t+1) W)
//    (W ~ 256 mean rows, at most 4096), so every tile carries about the same
//    number of nonzeros;
//    phase 1 streams the tile's column indices and values with coalesced
//    loads, forms a_ij * g(x_j) for every nonzero (eight gathers in flight
//    per thread) and parks the products in LDS; phase 2 lets `lpr` lanes per
//    row add them up and runs the row's epilogue.  Used whenever the longest
//    row fits the LDS reserve (every matrix of the workloads here).  Tiles
//    of long rows load the next tile during phase 2.
//  - vector: `lpr` lanes walk each row directly (rows too long for a tile).
// Blocks are renumbered so that each XCD owns one contiguous slab of rows
// (its L2 then serves the gathered vector entries those rows share).
//
// Reductions are deterministic and fence-free: a producing kernel writes one
// partial per block; the consuming kernel (one kernel later in the stream)
// adds the partials in index order in every block that needs the total.
// Scalars of the recurrence stay in device memory; once the stopping test
// passes, every later kernel sees `done` and returns at once.
#include <hip/hip_ext.h>

#include "devutil.hpp"
#include "internal.hpp"

namespace camg {

namespace {

#ifndef CAMG_TILE_W
#define CAMG_TILE_W 2048
#endif
#ifndef CAMG_TILE_ROWS
#define CAMG_TILE_ROWS 128
#endif
constexpr int kTileW = CAMG_TILE_W;        // largest nominal nonzeros per tile
constexpr int kTileRows = CAMG_TILE_ROWS;  // nominal rows per tile
constexpr int kTileMaxRow = 4096; // longest row a tile can hold (LDS <= 8192 entries)
constexpr int kTileWLong = 1664;   // nominal nonzeros per tile of the pipelined (long-row) loop
// Blocks of a row kernel: up to four times the 2048 a round of eight waves
// per SIMD holds, so blocks that finish early are replaced and the last
// round stays short (FP64 kernels and long rows measured 3-6 % faster with
// 8192 than with 2048); FP32 kernels of short rows move so few bytes per
// tile that the extra blocks' start-up and partial sums cost more than they
// balance, and keep 2048.
constexpr int kMaxRowGrid = 8192;
constexpr int kMaxRowGridShort32 = 2048;
static_assert(kMaxRowGrid <= kMaxPartials, "row-kernel partials would overflow");

template <class T>
struct MatArg {
    const int32_t *__restrict__ rp;
    const int32_t *__restrict__ ci;
    const T *__restrict__ v;
    const int32_t *__restrict__ tstart;  // tile mode: first row of each tile (ntiles + 1)
    const int32_t *__restrict__ tbase;   // tile mode with compact columns: kTileWins window starts per tile
    const uint16_t *__restrict__ off;    //   and the 16-bit word per nonzero (null: use ci)
    int off_mode;                        //   1: column = first start + word; 2: window in the top bits
    int n;
    int rpt;     // vector mode: rows per block
    int ntiles;  // tile mode
    int tpb;     // tiles per block
    int junk;    // tile mode: spare LDS slot after the tile
};

template <class T>
static const T *vals(const Csr &A);
template <>
const double *vals<double>(const Csr &A) { return A.v; }
template <>
const float *vals<float>(const Csr &A) { return A.v32; }

template <class T>
MatArg<T> mat_arg(const Csr &A, const RowCfg &c, const T *v = nullptr) {
    return MatArg<T>{A.rp,        A.ci,  v ? v : vals<T>(A), c.tstart, c.use_off ? c.tbase : nullptr,
                     c.use_off ? c.off : nullptr, c.off_mode, A.nr, c.rpt, c.ntiles, c.tpb, c.tile_nnz};
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

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned short v4us __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Positions, from the start of a step of 4*kBlock nonzeros, of the four
// nonzeros a thread takes.  FP32: four consecutive ones (one 16-byte load per
// thread, so a wavefront's load covers one contiguous KiB).  FP64: two pairs
// 2*kBlock apart, again one contiguous KiB per wavefront and load (four
// consecutive doubles per thread would take two loads that each leave half
// of every cache line they touch to the other; such loads measured 13 %
// slower on 7-point rows).
template <class T>
__device__ __forceinline__ int quad_pos(int u) {
    if constexpr (sizeof(T) == 4) return 4 * (int)threadIdx.x + u;
    else return 2 * (int)threadIdx.x + (u & 1) + (u >> 1) * (2 * kBlock);
}

// The column words (as stored) and values of this thread's four nonzeros in
// the step that starts s entries after a0 (a0 a multiple of 4).  A group that
// starts at or past `span` reads the tile's first entries instead (inside the
// arrays, no branch); the caller sends its products to the junk slot.  The
// arrays carry 8 elements of padding, so a group that starts inside the span
// stays inside the allocation.
template <int MODE, class T>
struct Quad {
    using W = std::conditional_t<MODE == 0, int, unsigned short>;
    W c[4];
    T v[4];
};
typedef int v2i __attribute__((ext_vector_type(2)));
typedef unsigned short v2us __attribute__((ext_vector_type(2)));
template <int MODE, class T>
__device__ __forceinline__ void fetch_quad(const MatArg<T> &M, int a0, int s, int span, Quad<MODE, T> &Q) {
    if constexpr (sizeof(T) == 4) {
        const int p = s + 4 * (int)threadIdx.x;
        const int idx = a0 + (p < span ? p : 0);
        const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(M.v + idx));
        Q.v[0] = v.x; Q.v[1] = v.y; Q.v[2] = v.z; Q.v[3] = v.w;
        if constexpr (MODE == 0) {
            const v4i c = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(M.ci + idx));
            Q.c[0] = c.x; Q.c[1] = c.y; Q.c[2] = c.z; Q.c[3] = c.w;
        } else {
            const v4us c = __builtin_nontemporal_load(reinterpret_cast<const v4us *>(M.off + idx));
            Q.c[0] = c.x; Q.c[1] = c.y; Q.c[2] = c.z; Q.c[3] = c.w;
        }
    } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = s + 2 * (int)threadIdx.x + h * (2 * kBlock);
            const int idx = a0 + (p < span ? p : 0);
            const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(M.v + idx));
            Q.v[2 * h] = v.x; Q.v[2 * h + 1] = v.y;
            if constexpr (MODE == 0) {
                const v2i c = __builtin_nontemporal_load(reinterpret_cast<const v2i *>(M.ci + idx));
                Q.c[2 * h] = c.x; Q.c[2 * h + 1] = c.y;
            } else {
                const v2us c = __builtin_nontemporal_load(reinterpret_cast<const v2us *>(M.off + idx));
                Q.c[2 * h] = c.x; Q.c[2 * h + 1] = c.y;
            }
        }
    }
}

// Column of a stored word: MODE 0 the int32 column; MODE 1 the tile's
// smallest column plus the 16-bit word; MODE 2 the start of the window named
// by the word's top bits (from LDS, wins) plus its low bits.
__device__ __forceinline__ int decode_col(const int *wins, unsigned o) {
    return wins[o >> kWinBits] + (int)(o & ((1u << kWinBits) - 1));
}
template <int MODE, class W>
__device__ __forceinline__ int word_col(W w, const int *wins, int base) {
    if constexpr (MODE == 0) return (int)w;
    else if constexpr (MODE == 1) return base + (int)w;
    else return decode_col(wins, w);
}

// prod[q] = a * g(col) for the four nonzeros of Q, q = position in the tile
// (entries outside [0, m) gather column 0 and store into prod[junk]).
template <int MODE, class T, class G>
__device__ __forceinline__ void park_quads(const G &g, T *prod, const Quad<MODE, T> *Q, int nq, int qs, int m,
                                           int junk, const int *wins, int base) {
    T gv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (u < 4 * nq) {
            const int q = qs + (u >> 2) * (4 * kBlock) + quad_pos<T>(u & 3);
            gv[u] = g((q >= 0 && q < m) ? word_col<MODE>(Q[u >> 2].c[u & 3], wins, base) : 0);
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (u < 4 * nq) {
            const int q = qs + (u >> 2) * (4 * kBlock) + quad_pos<T>(u & 3);
            prod[(q >= 0 && q < m) ? q : junk] = Q[u >> 2].v[u & 3] * gv[u];
        }
    }
}

// Phase 1 of a tile: prod[e - e0] = a_e * g(col_e) for e in [e0, e0 + m),
// streamed from e0 rounded down to a multiple of 4, two steps at a time
// (eight gathers in flight per thread), with no branch around the loads.
template <int MODE, class T, class G>
__device__ __forceinline__ void stream_tile(const MatArg<T> &M, const G &g, T *prod, int e0, int m,
                                            const int *wins, int base) {
    const int a0 = e0 & ~3;
    const int span = e0 + m - a0;
    constexpr int STEP = 4 * kBlock;
    int s = 0;
    for (; s + STEP < span; s += 2 * STEP) {
        Quad<MODE, T> Q[2];
        fetch_quad<MODE>(M, a0, s, span, Q[0]);
        fetch_quad<MODE>(M, a0, s + STEP, span, Q[1]);
        park_quads<MODE>(g, prod, Q, 2, a0 + s - e0, m, M.junk, wins, base);
    }
    if (s < span) {
        Quad<MODE, T> Q[1];
        fetch_quad<MODE>(M, a0, s, span, Q[0]);
        park_quads<MODE>(g, prod, Q, 1, a0 + s - e0, m, M.junk, wins, base);
    }
}

// Scalar variant of phase 1 for gathers that read two vectors per nonzero
// (fewer registers than the vector variant, so more waves stay resident).
template <class T, class G>
__device__ __forceinline__ void stream_tile_scalar(const MatArg<T> &M, const G &g, T *prod, int e0, int m) {
    int k = threadIdx.x;
    for (; k + 7 * kBlock < m; k += 8 * kBlock) {
        int j[8];
        T a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) j[u] = M.ci[e0 + k + u * kBlock];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = M.v[e0 + k + u * kBlock];
#pragma unroll
        for (int u = 0; u < 8; ++u) prod[k + u * kBlock] = a[u] * g(j[u]);
    }
    for (; k + 3 * kBlock < m; k += 4 * kBlock) {
        int j[4];
        T a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) j[u] = M.ci[e0 + k + u * kBlock];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = M.v[e0 + k + u * kBlock];
#pragma unroll
        for (int u = 0; u < 4; ++u) prod[k + u * kBlock] = a[u] * g(j[u]);
    }
    for (; k < m; k += kBlock) prod[k] = M.v[e0 + k] * g(M.ci[e0 + k]);
}

// Phase 1 split in two for a pipelined tile loop: tile_fetch issues the
// loads of the first two steps of a tile into registers (the column words as
// stored, so nothing waits on them), tile_consume gathers, multiplies and
// parks the products, then streams whatever lies beyond the two steps as
// stream_tile does.
template <int MODE, class T>
struct TileRegs {
    Quad<MODE, T> q[2];
};
template <int MODE, class T>
__device__ __forceinline__ void tile_fetch(const MatArg<T> &M, TileRegs<MODE, T> &R, int e0, int m) {
    const int a0 = e0 & ~3, span = e0 + m - a0;
    fetch_quad<MODE>(M, a0, 0, span, R.q[0]);
    fetch_quad<MODE>(M, a0, 4 * kBlock, span, R.q[1]);
}
template <int MODE, class T, class G>
__device__ __forceinline__ void tile_consume(const MatArg<T> &M, const G &g, T *prod, const TileRegs<MODE, T> &R,
                                             int e0, int m, int base) {
    const int a0 = e0 & ~3;
    const int span = e0 + m - a0;
    constexpr int STEP = 4 * kBlock;
    park_quads<MODE>(g, prod, R.q, 2, a0 - e0, m, M.junk, nullptr, base);
    for (int s = 2 * STEP; s < span; s += STEP) {
        Quad<MODE, T> Q[1];
        fetch_quad<MODE>(M, a0, s, span, Q[0]);
        park_quads<MODE>(g, prod, Q, 1, a0 + s - e0, m, M.junk, nullptr, base);
    }
}

// The tile loop of SHAPE 1 with the next tile's matrix loads issued before
// the current tile's row sums, so they travel while phase 2 runs.  The
// products and their order of summation are those of run_rows.
template <class T, int LPR, int MODE, class G, class E>
__device__ __forceinline__ void run_tiles_pipelined(const MatArg<T> &M, const G &g, const E &epi, T *prod,
                                                    double &dot) {
    const int sl = threadIdx.x & (LPR - 1), grp = threadIdx.x / LPR;
    constexpr int RPP = kBlock / LPR;
    using Pre = typename E::Pre;
    const int b = xcd_block();
    const int t0 = (int)((int64_t)b * M.ntiles / gridDim.x);
    const int t1 = (int)((int64_t)(b + 1) * M.ntiles / gridDim.x);
    if (t0 >= t1) return;
    int r0 = M.tstart[t0], r1 = M.tstart[t0 + 1];
    int e0 = M.rp[r0], m = M.rp[r1] - e0;
    TileRegs<MODE, T> R;
    tile_fetch<MODE>(M, R, e0, m);
    for (int t = t0; t < t1; ++t) {
        // the next tile's bounds, needed where its loads are issued
        const int nr1 = t + 1 < t1 ? M.tstart[t + 2] : r1;
        const int ne0 = M.rp[r1], nm = M.rp[nr1] - ne0;
        const int base = MODE == 1 ? M.tbase[(size_t)t * kTileWins] : 0;
        // every lane loads its row's bounds and epilogue operands (a valid
        // row where it has none), so no branch sits between these loads and
        // the gathers: the gathers then wait only for the prefetched words
        const int i = r0 + grp;
        const bool has = i < r1;
        const int ic = has ? i : (r1 > 0 ? r1 - 1 : 0);
        const int qa = M.rp[ic] - e0, qz = M.rp[ic + 1] - e0;
        const Pre pre = epi.load(ic);
        tile_consume<MODE>(M, g, prod, R, e0, m, base);
        __syncthreads();
        if (t + 1 < t1) tile_fetch<MODE>(M, R, ne0, nm);
        {
            T acc = 0;
            if (has)
                for (int q = qa + sl; q < qz; q += LPR) acc += prod[q];
            acc = group_sum<LPR>(acc);
            if (has && sl == 0) epi.finish(i, acc, pre, dot);
        }
        for (int ib = r0 + RPP; ib < r1; ib += RPP) {
            const int i2 = ib + grp;
            T acc = 0;
            if (i2 < r1) {
                const int a2 = M.rp[i2] - e0, z2 = M.rp[i2 + 1] - e0;
                for (int q = a2 + sl; q < z2; q += LPR) acc += prod[q];
            }
            acc = group_sum<LPR>(acc);
            if (i2 < r1 && sl == 0) epi.finish(i2, acc, epi.load(i2), dot);
        }
        __syncthreads();
        r0 = r1;
        r1 = nr1;
        e0 = ne0;
        m = nm;
    }
}

// Walk this block's rows; for each row i call
//   epi.finish(i, sum_j a_ij g(j), epi.load(i), dot).
// In tile mode the first row a lane group owns has its row pointers and its
// epilogue operands loaded before phase 1, so those loads overlap the
// streaming of the tile; phase 2 then only touches LDS and the output.
// SHAPE 0: vector rows; 1: tiles with int32 or one-base compact columns;
// 2: tiles with windowed compact columns (a separate kernel, so the other
// shapes keep their register budget)
template <class T, int LPR, int SHAPE, class G, class E>
__device__ __forceinline__ void run_rows(const MatArg<T> &M, const G &g, const E &epi, T *prod, double &dot) {
    const int sl = threadIdx.x & (LPR - 1), grp = threadIdx.x / LPR;
    constexpr int RPP = kBlock / LPR;  // rows per pass
    using Pre = typename E::Pre;
    // Tiles of long rows (eight and more lanes per row): the next tile's
    // loads overlap the current tile's row sums (short-row tiles measured no
    // gain).
    if constexpr (SHAPE == 1 && G::kLoads == 1 && LPR >= 8) {
        if (M.off) run_tiles_pipelined<T, LPR, 1>(M, g, epi, prod, dot);
        else run_tiles_pipelined<T, LPR, 0>(M, g, epi, prod, dot);
        return;
    }
    if constexpr (SHAPE > 0) {
        const int b = xcd_block();
        const int t0 = (int)((int64_t)b * M.ntiles / gridDim.x);
        const int t1 = (int)((int64_t)(b + 1) * M.ntiles / gridDim.x);
        __shared__ int wins[kTileWins];  // compact columns: this tile's window starts
        for (int t = t0; t < t1; ++t) {
            const int r0 = M.tstart[t], r1 = M.tstart[t + 1];
            if (r0 == r1) continue;
            const int e0 = M.rp[r0], m = M.rp[r1] - e0;
            if constexpr (SHAPE == 2) {  // the previous tile's readers passed the barrier that ended it
                if (threadIdx.x < kTileWins) wins[threadIdx.x] = M.tbase[(size_t)t * kTileWins + threadIdx.x];
                __syncthreads();
            }
            const int i = r0 + grp;
            const bool has = i < r1;
            int qa = 0, qz = 0;
            Pre pre{};
            if (has) {
                qa = M.rp[i] - e0;
                qz = M.rp[i + 1] - e0;
                if (sl == 0) pre = epi.load(i);
            }
            if constexpr (G::kLoads > 1) stream_tile_scalar(M, g, prod, e0, m);
            else if constexpr (SHAPE == 2) stream_tile<2>(M, g, prod, e0, m, wins, 0);
            else if (M.off) stream_tile<1>(M, g, prod, e0, m, wins, M.tbase[(size_t)t * kTileWins]);
            else stream_tile<0>(M, g, prod, e0, m, wins, 0);
            __syncthreads();
            {
                T acc = 0;
                for (int q = qa + sl; q < qz; q += LPR) acc += prod[q];
                acc = group_sum<LPR>(acc);
                if (has && sl == 0) epi.finish(i, acc, pre, dot);
            }
            for (int ib = r0 + RPP; ib < r1; ib += RPP) {
                const int i2 = ib + grp;
                T acc = 0;
                if (i2 < r1) {
                    const int a2 = M.rp[i2] - e0, z2 = M.rp[i2 + 1] - e0;
                    for (int q = a2 + sl; q < z2; q += LPR) acc += prod[q];
                }
                acc = group_sum<LPR>(acc);
                if (i2 < r1 && sl == 0) epi.finish(i2, acc, epi.load(i2), dot);
            }
            __syncthreads();
        }
    } else {
        const int b = xcd_block();
        const int r0 = (int)((int64_t)b * M.n / gridDim.x);
        const int r1 = (int)((int64_t)(b + 1) * M.n / gridDim.x);
        for (int ib = r0; ib < r1; ib += RPP) {
            const int i = ib + grp;
            T acc = 0;
            if (i < r1) {
                const int e1 = M.rp[i + 1];
                for (int e = M.rp[i] + sl; e < e1; e += LPR) acc += M.v[e] * g(M.ci[e]);
            }
            acc = group_sum<LPR>(acc);
            if (i < r1 && sl == 0) epi.finish(i, acc, epi.load(i), dot);
        }
    }
}

// ------------------------------------------------------------------ gathers and epilogues
template <class T, class TY>
struct GPre {  // s_j of the first Jacobi step from s = 0
    static constexpr int kLoads = 2;
    const T *wd;
    const TY *y;
    __device__ T operator()(int j) const { return wd[j] * (T)y[j]; }
};
template <class T, class TX = T>
struct GVec {
    static constexpr int kLoads = 1;
    const TX *x;
    __device__ T operator()(int j) const { return (T)x[j]; }
};
// The new search direction p = z + beta p_old, formed on the fly.  On the
// first iteration (and after a restart) beta = 0 and p_old is finite, so
// z + 0 * p_old is exactly z: no branch is needed.
template <class T, class TY>
struct EPre {  // s = wd y, r = y - A s
    const T *wd;
    const TY *y;
    T *s, *r;
    struct Pre {
        T yi, wdi;
    };
    __device__ Pre load(int i) const { return Pre{(T)y[i], wd[i]}; }
    __device__ void finish(int i, T acc, const Pre &p, double &) const {
        s[i] = p.wdi * p.yi;
        r[i] = p.yi - acc;
    }
};
template <class T, class TY, class TZ>
struct EPost {  // z = s + wd (y - A s); dot += y.z
    const T *wd;
    const TY *y;
    const T *s;
    TZ *z;
    struct Pre {
        TY yo;
        T wdi, si;
    };
    __device__ Pre load(int i) const { return Pre{y[i], wd[i], s[i]}; }
    __device__ void finish(int i, T acc, const Pre &p, double &dot) const {
        const T zi = p.si + p.wdi * ((T)p.yo - acc);
        const TZ zo = (TZ)zi;
        z[i] = zo;
        dot += (double)p.yo * (double)zo;
    }
};
template <class T, class TY>
struct EResid {  // r = y - A s
    const TY *y;
    T *r;
    struct Pre {
        T yi;
    };
    __device__ Pre load(int i) const { return Pre{(T)y[i]}; }
    __device__ void finish(int i, T acc, const Pre &p, double &) const { r[i] = p.yi - acc; }
};
template <class T, bool ADD>
struct ESpmv {
    T *out;
    struct Pre {
        T o;
    };
    __device__ Pre load(int i) const { return Pre{ADD ? out[i] : T(0)}; }
    __device__ void finish(int i, T acc, const Pre &p, double &) const { out[i] = ADD ? p.o + acc : acc; }
};
template <class T>
struct EScale {  // out = omega * (A x)  (first FSAI step: s = omega G^T u)
    T omega;
    T *out;
    struct Pre {};
    __device__ Pre load(int) const { return Pre{}; }
    __device__ void finish(int i, T acc, const Pre &, double &) const { out[i] = omega * acc; }
};
template <class T, class TY, class TZ>
struct EAddScaled {  // z = s + omega (A x); dot += y.z when y is given  (FSAI step; z may be s)
    T omega;
    const T *s;
    const TY *y;
    TZ *z;
    struct Pre {
        T si;
    };
    __device__ Pre load(int i) const { return Pre{s[i]}; }
    __device__ void finish(int i, T acc, const Pre &p, double &dot) const {
        const TZ zo = (TZ)(p.si + omega * acc);
        z[i] = zo;
        if (y) dot += (double)y[i] * (double)zo;
    }
};
struct EPQ {  // q = A p; dot += p.q
    const double *p;
    double *q;
    struct Pre {
        double pi;
    };
    __device__ Pre load(int i) const { return Pre{p[i]}; }
    __device__ void finish(int i, double acc, const Pre &pr, double &dot) const {
        q[i] = acc;
        dot += pr.pi * acc;
    }
};
struct EResNorm {  // d = b - A x; dot += d^2; optionally store d
    const double *b;
    double *out;
    struct Pre {
        double bi;
    };
    __device__ Pre load(int i) const { return Pre{b[i]}; }
    __device__ void finish(int i, double acc, const Pre &p, double &dot) const {
        const double d = p.bi - acc;
        if (out) out[i] = d;
        dot += d * d;
    }
};

// ------------------------------------------------------------------ kernels
// Waves per SIMD: eight, except for the pipelined FP64 tile loop, whose
// prefetched values take 16 more registers; at eight waves it would spill,
// at six it does not (and measured faster than the plain loop at eight).
template <class T, int LPR, int SHAPE, class G>
constexpr int kWaves = (sizeof(T) == 8 && SHAPE == 1 && LPR >= 8 && G::kLoads == 1) ? 6 : 8;
template <class T, int LPR, int SHAPE, bool DOT, class G, class E>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWaves<T, LPR, SHAPE, G>, kWaves<T, LPR, SHAPE, G>))) k_rows(MatArg<T> M, G g, E e, double *partials, int32_t *nout,
                                                 const PcgState *st) {
    if (st && st->done) return;
    extern __shared__ double smem_d[];
    T *prod = reinterpret_cast<T *>(smem_d);
    double dot = 0.0;
    run_rows<T, LPR, SHAPE>(M, g, e, prod, dot);
    if (DOT) {
        const double b = block_sum<kBlock>(dot);
        if (threadIdx.x == 0) {
            partials[blockIdx.x] = b;
            if (nout && blockIdx.x == 0) *nout = gridDim.x;
        }
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
                                                double *partials, int32_t *nout, const PcgState *st) {
    if (st && st->done) return;
    double acc = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) acc += y[i] * z[i];
    const double b = block_sum<kBlock>(acc);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = b;
        if (nout && blockIdx.x == 0) *nout = gridDim.x;
    }
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
            st->n_r2 = gridDim.x;
            st->n_rz = 0;
            st->n_pq = 0;
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
__global__ void __launch_bounds__(kBlock) k_pcg_check(const double *pr2, PcgState *st, double *hist, int hist_cap,
                                                      int32_t *hflag) {
    if (st->done) return;
    const double rn = sqrt(sum_all(pr2, st->n_r2));
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

// The vector kernels below need a scalar that every block sums from the
// partials of the kernel before (thousands of them); each thread first
// issues the loads of its first kVecAhead elements, so their latency
// overlaps that sum.  Elements are visited in the same order either way.
constexpr int kVecAhead = 4;

// rho = sum of the post-smoothing partials, beta = rho / rho_old (0 on a
// (re)start); p_new = z + beta p_old, streamed
__global__ void __launch_bounds__(kBlock) k_pcg_pnew(int n, const double *__restrict__ z,
                                                     const double *__restrict__ pold, double *__restrict__ pnew,
                                                     const double *prz, PcgState *st) {
    if (st->done) return;
    const int stride = gridDim.x * kBlock, i0 = blockIdx.x * kBlock + threadIdx.x;
    double za[kVecAhead], pa[kVecAhead];
#pragma unroll
    for (int u = 0; u < kVecAhead; ++u) {
        const int i = i0 + u * stride;
        za[u] = i < n ? z[i] : 0.0;
        pa[u] = i < n ? pold[i] : 0.0;
    }
    const double rho = sum_all(prz, st->n_rz);
    const bool first = st->iter == st->restart;
    const double beta = first ? 0.0 : rho / st->rho_old;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho = rho;
        st->beta = beta;
    }
#pragma unroll
    for (int u = 0; u < kVecAhead; ++u) {
        const int i = i0 + u * stride;
        if (i < n) pnew[i] = za[u] + beta * pa[u];
    }
    for (int i = i0 + kVecAhead * stride; i < n; i += stride) pnew[i] = z[i] + beta * pold[i];
}

// sigma = sum of the p.q partials; breakdown test; alpha = rho / sigma;
// x += alpha p, r -= alpha q; partials of ||r||^2
__global__ void __launch_bounds__(kBlock) k_pcg_update(int n, const double *__restrict__ p,
                                                       const double *__restrict__ q, double *__restrict__ x,
                                                       double *__restrict__ r, const double *ppq, double *pr2,
                                                       PcgState *st, int32_t *hflag) {
    if (st->done) return;
    const int stride = gridDim.x * kBlock, i0 = xcd_block() * kBlock + threadIdx.x;
    double xa[kVecAhead], pa[kVecAhead], ra[kVecAhead], qa[kVecAhead];
#pragma unroll
    for (int u = 0; u < kVecAhead; ++u) {
        const int i = i0 + u * stride;
        const bool in = i < n;
        xa[u] = in ? x[i] : 0.0;
        pa[u] = in ? p[i] : 0.0;
        ra[u] = in ? r[i] : 0.0;
        qa[u] = in ? q[i] : 0.0;
    }
    const double sigma = sum_all(ppq, st->n_pq);
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
#pragma unroll
    for (int u = 0; u < kVecAhead; ++u) {
        const int i = i0 + u * stride;
        if (i < n) {
            x[i] = xa[u] + alpha * pa[u];
            const double ri = ra[u] - alpha * qa[u];
            r[i] = ri;
            acc += ri * ri;
        }
    }
    for (int i = i0 + kVecAhead * stride; i < n; i += stride) {
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
            st->n_r2 = gridDim.x;
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

// events that the next row-kernel launch of this host thread records at its
// own start and end (set by time_next_row_launch, cleared by that launch)
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

template <class T, bool DOT, class G, class E>
void launch_rows(const Csr &A, const RowCfg &c, const G &g, const E &e, double *partials, int32_t *nout,
                 const PcgState *st, hipStream_t s, const T *values = nullptr) {
    const MatArg<T> M = mat_arg<T>(A, c, values);
    const size_t smem = c.tile ? (size_t)(c.tile_nnz + 1) * sizeof(T) : 0;
    const int shape = !c.tile ? 0 : (M.off && M.off_mode == 2) ? 2 : 1;
    const int grid = sizeof(T) == 4 && c.lpr < 8 ? std::min(c.grid, kMaxRowGridShort32) : c.grid;
    if (t_ev_start) {  // timed launch: the events bracket the kernel's execution
        hipEvent_t a = t_ev_start, b = t_ev_stop;
        t_ev_start = t_ev_stop = nullptr;
        const dim3 gr(grid), bl(kBlock);
        const uint32_t sm = (uint32_t)smem;
        if (shape == 1) {
            CAMG_LPR_SWITCH(c.lpr, (hipExtLaunchKernelGGL(k_rows<T, L, 1, DOT, G, E>, gr, bl, sm, s, a, b, 0, M, g, e,
                                                          partials, nout, st)));
        } else if (shape == 2) {
            CAMG_LPR_SWITCH(c.lpr, (hipExtLaunchKernelGGL(k_rows<T, L, 2, DOT, G, E>, gr, bl, sm, s, a, b, 0, M, g, e,
                                                          partials, nout, st)));
        } else {
            CAMG_LPR_SWITCH(c.lpr, (hipExtLaunchKernelGGL(k_rows<T, L, 0, DOT, G, E>, gr, bl, sm, s, a, b, 0, M, g, e,
                                                          partials, nout, st)));
        }
        HIPC(hipGetLastError());
        return;
    }
    if (shape == 1) {
        CAMG_LPR_SWITCH(c.lpr, (k_rows<T, L, 1, DOT, G, E><<<grid, kBlock, smem, s>>>(M, g, e, partials, nout, st)));
    } else if (shape == 2) {
        CAMG_LPR_SWITCH(c.lpr, (k_rows<T, L, 2, DOT, G, E><<<grid, kBlock, smem, s>>>(M, g, e, partials, nout, st)));
    } else {
        CAMG_LPR_SWITCH(c.lpr, (k_rows<T, L, 0, DOT, G, E><<<grid, kBlock, 0, s>>>(M, g, e, partials, nout, st)));
    }
    HIPC(hipGetLastError());
}

}  // namespace

void time_next_row_launch(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}

bool cancel_row_launch_timing() {
    const bool pending = t_ev_start != nullptr;
    t_ev_start = t_ev_stop = nullptr;
    return pending;
}

RowCfg choose_cfg(int n, int64_t nnz, int maxrow) {
    RowCfg c;
    const double mean = n > 0 ? std::max(1.0, (double)nnz / n) : 1.0;
    c.maxrow = maxrow;
    if (maxrow <= kTileMaxRow) {
        // about kTileRows rows per tile, at most kTileW nonzeros
        int W = (int)std::min<double>(kTileW, std::max(256.0, kTileRows * mean));
        W = (W + 63) / 64 * 64;
        auto lanes = [&](int w) {
            const double rows = w / mean;
            int l = 1;
            while (l * 2 <= 64 && l * 2 * rows <= kBlock) l *= 2;
            return l;
        };
        // tiles of the pipelined loop (eight and more lanes per row) hold
        // kTileWLong nominal nonzeros, so that a tile with its last row's
        // overhang mostly stays within the two prefetched steps of
        // 4 * kBlock entries
        if (lanes(W) >= 8) W = std::min(W, kTileWLong);
        c.tile = true;
        c.W = W;
        c.tile_nnz = W + std::max(maxrow, 1);
        c.lpr = lanes(W);
        c.ntiles = (int)std::max<int64_t>(1, (nnz + W - 1) / W);
        int g = std::min(c.ntiles, kMaxRowGrid);
        g = std::max(8, (g + 7) / 8 * 8);
        c.grid = g;
        c.tpb = (c.ntiles + g - 1) / g;
        c.rpt = 0;
    } else {
        c.tile = false;
        c.lpr = 64;
        const int rpp = kBlock / c.lpr;
        int g = (n + rpp - 1) / rpp;
        g = std::min(g, kMaxRowGrid);
        g = std::max(8, (g + 7) / 8 * 8);
        c.grid = g;
        const int per = (n + g - 1) / g;
        c.rpt = (per + rpp - 1) / rpp * rpp;
        c.ntiles = 0;
        c.tpb = 0;
        c.tile_nnz = 0;
    }
    return c;
}

int vec_grid(int n) {
    int g = std::min(kMaxGrid, std::max(8, (n + kBlock - 1) / kBlock));
    return (g + 7) / 8 * 8;
}

template <class T, class TY>
void vc_pre(const Csr &A, const RowCfg &c, const T *wd, const T *awd, const TY *y, T *s, T *r, const PcgState *st,
            hipStream_t str) {
    if (awd)  // values pre-scaled by wd_j: one gather per nonzero
        launch_rows<T, false>(A, c, GVec<T, TY>{y}, EPre<T, TY>{wd, y, s, r}, nullptr, nullptr, st, str, awd);
    else
        launch_rows<T, false>(A, c, GPre<T, TY>{wd, y}, EPre<T, TY>{wd, y, s, r}, nullptr, nullptr, st, str);
}

template <class T, class TY, class TZ, bool DOT>
void vc_post(const Csr &A, const RowCfg &c, const T *wd, const TY *y, const T *s, TZ *z, double *partials,
             int32_t *nout, const PcgState *st, hipStream_t str) {
    launch_rows<T, DOT>(A, c, GVec<T>{s}, EPost<T, TY, TZ>{wd, y, s, z}, partials, nout, st, str);
}

template <class T, class TY>
void vc_resid(const Csr &A, const RowCfg &c, const TY *y, const T *s, T *r, const PcgState *st, hipStream_t str) {
    launch_rows<T, false>(A, c, GVec<T>{s}, EResid<T, TY>{y, r}, nullptr, nullptr, st, str);
}

template <class T>
void vc_restrict(const Csr &R, const RowCfg &c, const T *r, T *yc, const PcgState *st, hipStream_t str) {
    launch_rows<T, false>(R, c, GVec<T>{r}, ESpmv<T, false>{yc}, nullptr, nullptr, st, str);
}

template <class T>
void vc_prolong(const Csr &P, const RowCfg &c, const T *d, T *s, const PcgState *st, hipStream_t str) {
    launch_rows<T, false>(P, c, GVec<T>{d}, ESpmv<T, true>{s}, nullptr, nullptr, st, str);
}

template <class T, class TY>
void vc_gmul(const Csr &G, const RowCfg &c, const TY *y, T *u, const PcgState *st, hipStream_t str) {
    launch_rows<T, false>(G, c, GVec<T, TY>{y}, ESpmv<T, false>{u}, nullptr, nullptr, st, str);
}

template <class T>
void vc_fsai_first(const Csr &Gt, const RowCfg &c, T omega, const T *u, T *s, const PcgState *st, hipStream_t str) {
    launch_rows<T, false>(Gt, c, GVec<T>{u}, EScale<T>{omega, s}, nullptr, nullptr, st, str);
}

template <class T, class TY, class TZ, bool DOT>
void vc_fsai_step(const Csr &Gt, const RowCfg &c, T omega, const T *u, const T *s, const TY *y, TZ *z,
                  double *partials, int32_t *nout, const PcgState *st, hipStream_t str) {
    launch_rows<T, DOT>(Gt, c, GVec<T>{u}, EAddScaled<T, TY, TZ>{omega, s, y, z}, partials, nout, st, str);
}

template <class T>
void coarse_solve(int n, const double *cinv, const T *y, T *z, const PcgState *st, hipStream_t str) {
    k_coarse<T><<<(n + 3) / 4, kBlock, 0, str>>>(n, cinv, y, z, st);
    HIPC(hipGetLastError());
}

#define INST_PRE(T, TY) template void vc_pre<T, TY>(const Csr &, const RowCfg &, const T *, const T *, const TY *, T *, \
                                                     T *, const PcgState *, hipStream_t);
INST_PRE(double, double)
INST_PRE(float, float)
INST_PRE(float, double)
#define INST_RES(T, TY) template void vc_resid<T, TY>(const Csr &, const RowCfg &, const TY *, const T *, T *, \
                                                       const PcgState *, hipStream_t);
INST_RES(double, double)
INST_RES(float, float)
INST_RES(float, double)
#define INST_POST(T, TY, TZ, D) template void vc_post<T, TY, TZ, D>(const Csr &, const RowCfg &, const T *, const TY *, \
                                                                     const T *, TZ *, double *, int32_t *, const PcgState *, \
                                                                     hipStream_t);
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
template void vc_gmul<double, double>(const Csr &, const RowCfg &, const double *, double *, const PcgState *,
                                      hipStream_t);
template void vc_gmul<float, float>(const Csr &, const RowCfg &, const float *, float *, const PcgState *, hipStream_t);
template void vc_gmul<float, double>(const Csr &, const RowCfg &, const double *, float *, const PcgState *,
                                     hipStream_t);
template void vc_fsai_first<double>(const Csr &, const RowCfg &, double, const double *, double *, const PcgState *,
                                    hipStream_t);
template void vc_fsai_first<float>(const Csr &, const RowCfg &, float, const float *, float *, const PcgState *,
                                   hipStream_t);
#define INST_FSTEP(T, TY, TZ, D)                                                                                  \
    template void vc_fsai_step<T, TY, TZ, D>(const Csr &, const RowCfg &, T, const T *, const T *, const TY *, TZ *, \
                                             double *, int32_t *, const PcgState *, hipStream_t);
INST_FSTEP(double, double, double, false)
INST_FSTEP(double, double, double, true)
INST_FSTEP(float, float, float, false)
INST_FSTEP(float, double, float, false)
INST_FSTEP(float, double, double, false)
INST_FSTEP(float, double, double, true)
template void coarse_solve<double>(int, const double *, const double *, double *, const PcgState *, hipStream_t);
template void coarse_solve<float>(int, const double *, const float *, float *, const PcgState *, hipStream_t);

int dot_partials(int n, const double *y, const double *z, double *partials, int32_t *nout, const PcgState *st,
                 hipStream_t s) {
    const int g = std::min(kMaxGrid, std::max(1, (n + kBlock - 1) / kBlock));
    k_dot<<<g, kBlock, 0, s>>>(n, y, z, partials, nout, st);
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

void pcg_check(const double *pr2, PcgState *st, double *hist, int hist_cap, int32_t *hflag, hipStream_t s) {
    k_pcg_check<<<1, kBlock, 0, s>>>(pr2, st, hist, hist_cap, hflag);
    HIPC(hipGetLastError());
}

// New search direction and q = A p: p_new is streamed by one kernel, then
// q = A p_new runs as a one-gather row kernel with the p.q partials (one
// gathered vector instead of two in a fused kernel, whose second gather
// costs more than the extra pass over z, p_old and p_new).
int pcg_dir(const Csr &A, const RowCfg &c, const double *z, const double *pold, double *pnew, double *q,
            const double *prz, double *ppq, PcgState *st, hipStream_t s) {
    k_pcg_pnew<<<vec_grid(A.nr), kBlock, 0, s>>>(A.nr, z, pold, pnew, prz, st);
    HIPC(hipGetLastError());
    launch_rows<double, true>(A, c, GVec<double>{pnew}, EPQ{pnew, q}, ppq, &st->n_pq, st, s);
    return c.grid;
}

int pcg_update(int n, const double *p, const double *q, double *x, double *r, const double *ppq, double *pr2,
               PcgState *st, int32_t *hflag, hipStream_t s) {
    const int g = vec_grid(n);
    k_pcg_update<<<g, kBlock, 0, s>>>(n, p, q, x, r, ppq, pr2, st, hflag);
    HIPC(hipGetLastError());
    return g;
}

void pcg_restart(PcgState *st, hipStream_t s) {
    k_pcg_restart<<<1, 1, 0, s>>>(st);
    HIPC(hipGetLastError());
}

int residual_norm(const Csr &A, const RowCfg &c, const double *b, const double *x, double *out, double *partials,
                  int32_t *nout, hipStream_t s) {
    launch_rows<double, true>(A, c, GVec<double>{x}, EResNorm{b, out}, partials, nout, nullptr, s);
    return c.grid;
}

void sum_to(const double *partials, int n, double *out, hipStream_t s) {
    k_sum_to<<<1, kBlock, 0, s>>>(partials, n, out);
    HIPC(hipGetLastError());
}

}  // namespace camg
