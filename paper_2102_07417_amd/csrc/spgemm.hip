// Sparse matrix-matrix product Z = X Y for the Galerkin operator
// A_c = P^T (A P) (eq. AcDef), row by row, one wavefront per output row.
//
//   1. product bound: prod_i = sum over k in row i of X of |row k of Y|;
//   2. symbolic pass: the distinct columns of row i are counted with an
//      open-addressing hash table in LDS (sized from prod_i, bins of rows);
//   3. scan of the counts gives Z's row pointer;
//   4. fill pass: the table is rebuilt, its keys sorted (bitonic, in LDS)
//      and written as Z's columns; each slot then maps its column to the
//      sorted position, and the values are accumulated there walking X's
//      row in ascending order -- for a fixed inner index k the wavefront's
//      lanes hold distinct columns, so every output entry receives its
//      products one at a time in ascending k, starting from 0.0.  The sums
//      are therefore rounded exactly as a sequential row-by-row product
//      with a dense accumulator rounds them.
// Rows whose table would not fit in LDS use the same code on tables in a
// global scratch buffer.  galerkin() forms R (A P), in chunks of coarse rows
// when A P would be large.
#include <algorithm>
#include <climits>
#include <vector>

#include "devutil.hpp"
#include "internal.hpp"

namespace camg {

namespace {

constexpr int kEmpty = -1;
constexpr int kWPB = 4;  // wavefronts per block for the binned kernels

#define WAVE_SYNC()                                         \
    do {                                                    \
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                    \
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
    } while (0)

__device__ __forceinline__ unsigned slot_of(int j, int ts) { return ((unsigned)j * 2654435761u) & (unsigned)(ts - 1); }

struct CsrView {
    const int32_t *rp, *ci;
    const double *v;
};

// prod[i] = number of products of row i of X Y, G lanes per row of X
template <int G>
__global__ void k_row_products(int nr, CsrView X, CsrView Y, int64_t *prod) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / G), sl = (int)(t & (G - 1));
    const int e0 = i < nr ? X.rp[i] : 0, e1 = i < nr ? X.rp[i + 1] : 0;
    long long p = 0;
    for (int e = e0 + sl; e < e1; e += G) {
        const int k = X.ci[e];
        p += Y.rp[k + 1] - Y.rp[k];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) p += __shfl_xor(p, o, G);
    if (i < nr && sl == 0) prod[i] = p;
}

// first and last column of every row (INT_MAX / -1 for an empty row)
__global__ void k_row_span(int nr, const int32_t *rp, const int32_t *ci, int32_t *lo, int32_t *hi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const bool any = rp[i] < rp[i + 1];
    lo[i] = any ? ci[rp[i]] : INT_MAX;
    hi[i] = any ? ci[rp[i + 1] - 1] : -1;
}

// rows [c0, c0 + m) of X as a matrix of their own, columns shifted by -f0
__global__ void k_slice_rows(int m, const int32_t *rp, int c0, int32_t *rp2) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r <= m) rp2[r] = rp[c0 + r] - rp[c0];
}

__global__ void k_shift_cols(int64_t ne, const int32_t *ci, int f0, int32_t *ci2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ne) ci2[e] = ci[e] - f0;
}

__global__ void k_offset_rp(int m, const int32_t *rp, int64_t base, int32_t *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r <= m) out[r] = (int32_t)(rp[r] + base);
}

// bin b holds rows with value <= lim[b] (and > lim[b-1]); the last bin is
// open.  Slots are taken per block: LDS counters first, then one global
// atomic per block and bin.
// Rows with at most kThrX entries of X and kThrP products are formed by one
// thread each (k_sym_thread / k_fill_thread) and left out of the bins.
// A thread's merge is a chain of dependent loads, hidden only when many
// rows run at once: products of fewer rows than kThrMinRows give every row
// a wavefront of the binned kernels instead (the same sums in the same
// order either way).  `thrp` is kThrP, or -1 when no row is a thread row.
constexpr int kThrX = 16;
constexpr int64_t kThrP = 256;
constexpr int kThrMinRows = 262144;

__device__ __forceinline__ bool thread_row(const CsrView &X, const int64_t *prod, int i, int64_t thrp) {
    return X.rp[i + 1] - X.rp[i] <= kThrX && prod[i] <= thrp;
}

__global__ void k_bin_rows(int nr, const int64_t *val, const int32_t *rpv, int nb, const int64_t *lim, int32_t *bcnt,
                           int32_t *brows, int stride, CsrView X, const int64_t *prod, int64_t thrp) {
    __shared__ int lcnt[8], lbase[8];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x < 8) lcnt[threadIdx.x] = 0;
    __syncthreads();
    int b = -1, off = 0;
    if (i < nr && !thread_row(X, prod, i, thrp)) {
        const int64_t x = val ? val[i] : (int64_t)(rpv[i + 1] - rpv[i]);
        b = 0;
        while (b < nb - 1 && x > lim[b]) ++b;
        off = atomicAdd(&lcnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < nb) lbase[threadIdx.x] = lcnt[threadIdx.x] ? atomicAdd(&bcnt[threadIdx.x], lcnt[threadIdx.x]) : 0;
    __syncthreads();
    if (b >= 0) brows[(int64_t)b * stride + lbase[b] + off] = i;
}

// One thread per short row: a merge of the rows of Y named by the row of X,
// by column.  For each output column the contributing rows are visited in
// ascending order of X's entries and their products added one at a time
// from 0.0 -- the order of the wavefront kernels.
template <bool FILL>
__global__ void __launch_bounds__(256) k_thread_rows(int nr, CsrView X, CsrView Y, const int64_t *prod, int64_t thrp,
                                                     int32_t *cnt, const int32_t *zrp, int32_t *zci, double *zv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr || !thread_row(X, prod, i, thrp)) return;
    const int e0 = X.rp[i], m = X.rp[i + 1] - e0;
    int pos[kThrX], end[kThrX], head[kThrX];
    double xv[kThrX];
    for (int q = 0; q < m; ++q) {
        const int k = X.ci[e0 + q];
        pos[q] = Y.rp[k];
        end[q] = Y.rp[k + 1];
        head[q] = pos[q] < end[q] ? Y.ci[pos[q]] : INT_MAX;
        xv[q] = X.v[e0 + q];
    }
    const int o = FILL ? zrp[i] : 0;
    int c = 0;
    for (;;) {
        int j = INT_MAX;
        for (int q = 0; q < m; ++q) j = head[q] < j ? head[q] : j;
        if (j == INT_MAX) break;
        double acc = 0.0;
        for (int q = 0; q < m; ++q) {
            if (head[q] != j) continue;
            if (FILL) acc = acc + xv[q] * Y.v[pos[q]];
            ++pos[q];
            head[q] = pos[q] < end[q] ? Y.ci[pos[q]] : INT_MAX;
        }
        if (FILL) {
            zci[o + c] = j;
            zv[o + c] = acc;
        }
        ++c;
    }
    if (!FILL) cnt[i] = c;
}

// Visit the products of row i of X Y in ascending order of X's entries e:
// for each e the lanes take the entries t of row k = X.ci[e] of Y; each
// product (j = Y.ci[t], x = X.v[e], y = Y.v[t]) first goes through
// tok = pre(j, x, y), the part whose order does not matter, then through
// post(tok, x, y), and step e's post calls finish (wavefront barrier)
// before step e+1's start (when ORDERED).  The entries of X's row (column,
// value, extent of Y's row) are loaded by all lanes at once, 64 at a time.
// Steps go in groups of four.  When each of a group's four Y rows has at
// most 16 entries, lane 16 d + t takes entry t of the group's step d, the
// pre calls of the four steps run at once and the post calls step by step;
// otherwise the group's steps run one at a time, the lanes taking the first
// 64 entries of the step's Y row (and the rest in further passes).  The
// loads of the next group (one entry per lane when it is packed, else the
// first 64 entries of each of its four Y rows) are issued while the current
// group runs, so a step rarely waits for memory.
constexpr int kAhead = 4;
template <bool ORDERED, class Pre, class Post>
__device__ __forceinline__ void for_products(int i, const CsrView &X, const CsrView &Y, int lane, Pre pre,
                                             Post post) {
    const int e0 = X.rp[i], e1 = X.rp[i + 1];
    const int dl = lane >> 4, tl = lane & 15;  // packed groups: step and entry of this lane
    for (int cb = e0; cb < e1; cb += kWave) {
        const int ne = min(kWave, e1 - cb);
        int yb = 0, yc = 0;
        double xv = 0.0;
        if (lane < ne) {
            const int k = X.ci[cb + lane];
            xv = X.v[cb + lane];
            yb = Y.rp[k];
            yc = Y.rp[k + 1] - yb;
        }
        // whether the group of steps q0 .. q0+3 is packed (the same on every lane)
        auto packed = [&](int q0) {
            int m = 0;
#pragma unroll
            for (int d = 0; d < kAhead; ++d) {
                const int q = q0 + d;
                const int c = __shfl(yc, q & (kWave - 1), kWave);
                if (q < ne) m = max(m, c);
            }
            return m <= 16;
        };
        // the loads of group q0: one entry per lane, or the first kWave
        // entries of each step's Y row
        auto load = [&](int q0, bool pk, int *jr, double *vr) {
#pragma unroll
            for (int d = 0; d < kAhead; ++d) {
                jr[d] = 0;
                vr[d] = 0.0;
            }
            if (pk) {
                const int q = q0 + dl;
                const int b = __shfl(yb, q & (kWave - 1), kWave), c = __shfl(yc, q & (kWave - 1), kWave);
                if (q < ne && tl < c) {
                    jr[0] = Y.ci[b + tl];
                    vr[0] = Y.v[b + tl];
                }
            } else {
#pragma unroll
                for (int d = 0; d < kAhead; ++d) {
                    const int q = q0 + d;
                    if (q < ne) {
                        const int b = __shfl(yb, q, kWave), c = __shfl(yc, q, kWave);
                        if (lane < c) {
                            jr[d] = Y.ci[b + lane];
                            vr[d] = Y.v[b + lane];
                        }
                    }
                }
            }
        };
        int jq[kAhead];
        double vq[kAhead];
        bool pk = packed(0);
        load(0, pk, jq, vq);
        for (int q0 = 0; q0 < ne; q0 += kAhead) {
            const bool more = q0 + kAhead < ne;
            const bool pkn = more ? packed(q0 + kAhead) : false;
            int jn[kAhead];
            double vn[kAhead];
            if (more) load(q0 + kAhead, pkn, jn, vn);
            if (pk) {
                const int q = q0 + dl;
                const int c = __shfl(yc, q & (kWave - 1), kWave);
                const double x = __shfl(xv, q & (kWave - 1), kWave);
                const bool act = q < ne && tl < c;
                int tok = 0;
                if (act) tok = pre(jq[0], x, vq[0]);
                if constexpr (ORDERED) {
#pragma unroll
                    for (int d = 0; d < kAhead; ++d) {
                        if (act && dl == d) post(tok, x, vq[0]);
                        WAVE_SYNC();
                    }
                } else {
                    WAVE_SYNC();
                }
            } else {
#pragma unroll
                for (int d = 0; d < kAhead; ++d) {
                    const int q = q0 + d;
                    if (q < ne) {
                        const int b = __shfl(yb, q, kWave), c = __shfl(yc, q, kWave);
                        const double x = __shfl(xv, q, kWave);
                        if (lane < c) post(pre(jq[d], x, vq[d]), x, vq[d]);
                        for (int t = b + kWave + lane; t < b + c; t += kWave) {
                            const int j = Y.ci[t];
                            const double y = Y.v[t];
                            post(pre(j, x, y), x, y);
                        }
                        WAVE_SYNC();
                    }
                }
            }
            pk = pkn;
#pragma unroll
            for (int d = 0; d < kAhead; ++d) {
                jq[d] = jn[d];
                vq[d] = vn[d];
            }
        }
    }
}

// Insert the columns of row i of X Y into the table; returns the number of
// new keys this lane inserted.  *overflow is set if a probe sequence wraps.
__device__ __forceinline__ int insert_row(int i, const CsrView &X, const CsrView &Y, int *keys, int ts, int lane,
                                          bool &overflow) {
    // the set of keys (and the count) does not depend on the order of the
    // insertions, so no step waits for the one before
    int cnt = 0;
    for_products<false>(
        i, X, Y, lane,
        [&](int j, double, double) {
            unsigned h = slot_of(j, ts);
            for (int probe = 0;; ++probe) {
                const int old = atomicCAS(&keys[h], kEmpty, j);
                if (old == kEmpty) {
                    ++cnt;
                    break;
                }
                if (old == j) break;
                h = (h + 1) & (unsigned)(ts - 1);
                if (probe >= ts) {
                    overflow = true;
                    break;
                }
            }
            return 0;
        },
        [](int, double, double) {});
    return cnt;
}

// slot holding key j (present by construction); -1 if absent after a full sweep
__device__ __forceinline__ int find_slot(const int *keys, int ts, int j) {
    unsigned h = slot_of(j, ts);
    for (int probe = 0; probe < ts; ++probe) {
        if (keys[h] == j) return (int)h;
        h = (h + 1) & (unsigned)(ts - 1);
    }
    return -1;
}

// ------------------------------------------------------------ symbolic
__device__ __forceinline__ void symbolic_row(int i, bool valid, const CsrView &X, const CsrView &Y, int *keys, int ts,
                                             int32_t *cnt_out, int32_t *ovf_flag) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int s = lane; s < ts; s += kWave) keys[s] = kEmpty;
    __syncthreads();
    bool overflow = false;
    int c = valid ? insert_row(i, X, Y, keys, ts, lane, overflow) : 0;
    c = wave_sum_i(c);
    const int ov = wave_sum_i(overflow ? 1 : 0);
    if (valid && lane == 0) {
        if (ov || c > (ts - ts / 4)) { cnt_out[i] = -1; atomicOr(ovf_flag, 1); }
        else cnt_out[i] = c;
    }
    __syncthreads();
}

template <int TS, int WPB>
__global__ void __launch_bounds__(WPB * 64) k_symbolic_lds(int nrows_bin, const int32_t *rows, CsrView X, CsrView Y,
                                                            int32_t *cnt, int32_t *ovf) {
    __shared__ int keys[WPB][TS];
    const int w = threadIdx.x / kWave;
    const int idx = blockIdx.x * WPB + w;
    const bool valid = idx < nrows_bin;
    const int i = valid ? rows[idx] : 0;
    symbolic_row(i, valid, X, Y, keys[w], TS, cnt, ovf);
}

// one wavefront per row, tables in global memory at offsets toff[idx]
__global__ void __launch_bounds__(64) k_symbolic_glb(int nrows, const int32_t *rows, const int64_t *toff,
                                                      const int32_t *tsz, CsrView X, CsrView Y, int *scratch,
                                                      int32_t *cnt, int32_t *ovf) {
    const int idx = blockIdx.x;
    if (idx >= nrows) return;
    symbolic_row(rows[idx], true, X, Y, scratch + toff[idx], tsz[idx], cnt, ovf);
}

// ------------------------------------------------------------ fill + numeric
__device__ __forceinline__ void fill_row(int i, bool valid, const CsrView &X, const CsrView &Y, const int32_t *zrp,
                                         int32_t *zci, double *zv, int *keys, int *pos, int *cols, double *acc,
                                         int ts, int *counter) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int s = lane; s < ts; s += kWave) keys[s] = kEmpty;
    if (lane == 0) *counter = 0;
    __syncthreads();
    bool overflow = false;
    if (valid) insert_row(i, X, Y, keys, ts, lane, overflow);
    __syncthreads();
    const int u = valid ? zrp[i + 1] - zrp[i] : 0;
    int npow = 1;
    while (npow < u) npow <<= 1;
    if (valid) {
        for (int s = lane; s < ts; s += kWave) {
            const int k = keys[s];
            if (k != kEmpty) {
                const int q = atomicAdd(counter, 1);
                if (q < npow) cols[q] = k;
            }
        }
        WAVE_SYNC();
        for (int p = u + lane; p < npow; p += kWave) cols[p] = INT_MAX;
        WAVE_SYNC();
        // bitonic sort of cols[0, npow)
        for (int kk = 2; kk <= npow; kk <<= 1) {
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int a = lane; a < npow; a += kWave) {
                    const int b = a ^ jj;
                    if (b > a) {
                        const int x = cols[a], y = cols[b];
                        const bool up = (a & kk) == 0;
                        if (up ? (x > y) : (x < y)) {
                            cols[a] = y;
                            cols[b] = x;
                        }
                    }
                }
                WAVE_SYNC();
            }
        }
        for (int p = lane; p < u; p += kWave) {
            const int h = find_slot(keys, ts, cols[p]);
            if (h >= 0) pos[h] = p;
            acc[p] = 0.0;
        }
        WAVE_SYNC();
        // products in ascending inner index; within a step the lanes hold
        // distinct columns
        for_products<true>(
            i, X, Y, lane,
            [&](int j, double, double) {
                const int h = find_slot(keys, ts, j);
                return h >= 0 ? pos[h] : -1;
            },
            [&](int p, double x, double y) {
                if (p >= 0) acc[p] = acc[p] + x * y;
            });
        const int off = zrp[i];
        for (int p = lane; p < u; p += kWave) {
            zci[off + p] = cols[p];
            zv[off + p] = acc[p];
        }
    }
    __syncthreads();
}

template <int TS, int UMAX, int WPB>
__global__ void __launch_bounds__(WPB * 64) k_fill_lds(int nrows_bin, const int32_t *rows, CsrView X, CsrView Y,
                                                        const int32_t *zrp, int32_t *zci, double *zv) {
    __shared__ int keys[WPB][TS];
    __shared__ int pos[WPB][TS];
    __shared__ int cols[WPB][UMAX];
    __shared__ double acc[WPB][UMAX];
    __shared__ int counter[WPB];
    const int w = threadIdx.x / kWave;
    const int idx = blockIdx.x * WPB + w;
    const bool valid = idx < nrows_bin;
    const int i = valid ? rows[idx] : 0;
    fill_row(i, valid, X, Y, zrp, zci, zv, keys[w], pos[w], cols[w], acc[w], TS, &counter[w]);
}

// global-table variant: scratch per row = keys[ts], pos[ts], cols[npow] (ints) and acc[u] (doubles)
__global__ void __launch_bounds__(64) k_fill_glb(int nrows, const int32_t *rows, const int64_t *ioff,
                                                  const int64_t *doff, const int32_t *tsz, CsrView X, CsrView Y,
                                                  const int32_t *zrp, int32_t *zci, double *zv, int *iscratch,
                                                  double *dscratch, int *counters) {
    const int idx = blockIdx.x;
    if (idx >= nrows) return;
    const int ts = tsz[idx];
    int *base = iscratch + ioff[idx];
    fill_row(rows[idx], true, X, Y, zrp, zci, zv, base, base + ts, base + 2 * ts, dscratch + doff[idx], ts,
             &counters[idx]);
}

inline int nblk(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// k_row_products with lanes per row matched to X's mean row length
void row_products(int nr, int64_t nnz, const CsrView &X, const CsrView &Y, int64_t *prod, hipStream_t s) {
    if (nr <= 0) return;
    const double mean = (double)nnz / nr;
    if (mean > 16) k_row_products<32><<<nblk((int64_t)nr * 32, kBlock), kBlock, 0, s>>>(nr, X, Y, prod);
    else if (mean > 4) k_row_products<8><<<nblk((int64_t)nr * 8, kBlock), kBlock, 0, s>>>(nr, X, Y, prod);
    else k_row_products<1><<<nblk(nr, kBlock), kBlock, 0, s>>>(nr, X, Y, prod);
    HIPC(hipGetLastError());
}

int next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return (int)p;
}

template <int TS, int WPB>
void launch_symbolic(int nb, const int32_t *rows, const CsrView &X, const CsrView &Y, int32_t *cnt, int32_t *ovf,
                     hipStream_t s) {
    if (nb <= 0) return;
    k_symbolic_lds<TS, WPB><<<nblk(nb, WPB), WPB * 64, 0, s>>>(nb, rows, X, Y, cnt, ovf);
    HIPC(hipGetLastError());
}

template <int TS, int UMAX, int WPB>
void launch_fill(int nb, const int32_t *rows, const CsrView &X, const CsrView &Y, const int32_t *zrp, int32_t *zci,
                 double *zv, hipStream_t s) {
    if (nb <= 0) return;
    k_fill_lds<TS, UMAX, WPB><<<nblk(nb, WPB), WPB * 64, 0, s>>>(nb, rows, X, Y, zrp, zci, zv);
    HIPC(hipGetLastError());
}

}  // namespace

void spgemm(const Csr &X, const Csr &Y, Csr &Z, Pool &out, Pool &tmp, hipStream_t s) {
    const int nr = X.nr;
    Z.nr = nr;
    Z.nc = Y.nc;
    Z.rp = out.alloc<int32_t>((size_t)nr + 1);
    if (nr == 0) {
        HIPC(hipMemsetAsync(Z.rp, 0, sizeof(int32_t), s));
        Z.nnz = 0;
        return;
    }
    CsrView xv{X.rp, X.ci, X.v}, yv{Y.rp, Y.ci, Y.v};

    // 1. product bounds and symbolic bins
    int64_t *prod = tmp.alloc<int64_t>(nr);
    row_products(nr, X.nnz, xv, yv, prod, s);

    constexpr int NB = 5;
    const int64_t sym_lim_h[NB] = {64, 256, 1024, 4096, INT64_MAX};
    int64_t *lim = tmp.alloc<int64_t>(NB);
    int32_t *bcnt = tmp.alloc<int32_t>(NB);
    int32_t *brows = tmp.alloc<int32_t>((size_t)NB * nr);
    int32_t *ovf = tmp.alloc<int32_t>(1);
    int32_t *cnt = tmp.alloc<int32_t>(nr);
    HIPC(hipMemcpyAsync(lim, sym_lim_h, sizeof(sym_lim_h), hipMemcpyHostToDevice, s));
    HIPC(hipMemsetAsync(bcnt, 0, sizeof(int32_t) * NB, s));
    HIPC(hipMemsetAsync(ovf, 0, sizeof(int32_t), s));
    const int64_t thrp = nr >= kThrMinRows ? kThrP : -1;
    k_bin_rows<<<nblk(nr, kBlock), kBlock, 0, s>>>(nr, prod, nullptr, NB, lim, bcnt, brows, nr, xv, prod, thrp);
    if (thrp >= 0)
        k_thread_rows<false><<<nblk(nr, 256), 256, 0, s>>>(nr, xv, yv, prod, thrp, cnt, nullptr, nullptr, nullptr);
    HIPC(hipGetLastError());
    int32_t hbs[NB];  // rows per symbolic bin
    HIPC(hipMemcpyAsync(hbs, bcnt, sizeof(hbs), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));

    // 2. symbolic
    launch_symbolic<128, kWPB>(hbs[0], brows + 0 * (size_t)nr, xv, yv, cnt, ovf, s);
    launch_symbolic<512, kWPB>(hbs[1], brows + 1 * (size_t)nr, xv, yv, cnt, ovf, s);
    launch_symbolic<2048, kWPB>(hbs[2], brows + 2 * (size_t)nr, xv, yv, cnt, ovf, s);
    launch_symbolic<8192, kWPB>(hbs[3], brows + 3 * (size_t)nr, xv, yv, cnt, ovf, s);
    launch_symbolic<16384, 2>(hbs[4], brows + 4 * (size_t)nr, xv, yv, cnt, ovf, s);
    // 3. row pointer, then the fill bins by exact row length; the overflow
    // flag, the product's size and the bin counts come back in one
    // read-back (the rare overflow path redoes the row pointer and bins)
    const int64_t fill_lim_h[NB] = {64, 256, 1024, 4096, INT64_MAX};
    int64_t *rp64 = tmp.alloc<int64_t>((size_t)nr + 1);
    int32_t *bcnt2 = tmp.alloc<int32_t>(NB);
    int32_t *brows2 = tmp.alloc<int32_t>((size_t)NB * nr);
    int64_t *flim = tmp.alloc<int64_t>(NB);
    HIPC(hipMemcpyAsync(flim, fill_lim_h, sizeof(fill_lim_h), hipMemcpyHostToDevice, s));
    int64_t nnz = 0;
    int32_t hovf = 0;
    int32_t hb[NB];  // rows per fill bin
    auto rowptr_and_bins = [&]() {
        scan_i32_to_i64(cnt, rp64, nr, tmp, s);
        narrow_i64(rp64, Z.rp, nr, s);  // checked against 2^31 - 1 below, before use
        HIPC(hipMemsetAsync(bcnt2, 0, sizeof(int32_t) * NB, s));
        k_bin_rows<<<nblk(nr, kBlock), kBlock, 0, s>>>(nr, nullptr, Z.rp, NB, flim, bcnt2, brows2, nr, xv, prod,
                                                       thrp);
        HIPC(hipGetLastError());
        HIPC(hipMemcpyAsync(&nnz, rp64 + nr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(&hovf, ovf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(hb, bcnt2, sizeof(hb), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
    };
    rowptr_and_bins();
    if (hovf) {
        // rows whose distinct columns overflowed the largest LDS table: redo
        // them with global tables sized from their product bound
        std::vector<int32_t> rows(hbs[4]);
        std::vector<int64_t> pr(nr);
        std::vector<int32_t> cn(nr);
        HIPC(hipMemcpy(rows.data(), brows + 4 * (size_t)nr, sizeof(int32_t) * rows.size(), hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(pr.data(), prod, sizeof(int64_t) * nr, hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(cn.data(), cnt, sizeof(int32_t) * nr, hipMemcpyDeviceToHost));
        std::vector<int32_t> grow, gts;
        std::vector<int64_t> goff;
        int64_t total = 0;
        for (int r : rows)
            if (cn[r] < 0) {
                const int ts = next_pow2(2 * pr[r] + 1);
                grow.push_back(r);
                gts.push_back(ts);
                goff.push_back(total);
                total += ts;
            }
        Pool g(s);
        int *scr = g.alloc<int>((size_t)total);
        int32_t *drows = g.alloc<int32_t>(grow.size());
        int32_t *dts = g.alloc<int32_t>(grow.size());
        int64_t *doff = g.alloc<int64_t>(grow.size());
        HIPC(hipMemcpyAsync(drows, grow.data(), sizeof(int32_t) * grow.size(), hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(dts, gts.data(), sizeof(int32_t) * grow.size(), hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(doff, goff.data(), sizeof(int64_t) * grow.size(), hipMemcpyHostToDevice, s));
        k_symbolic_glb<<<(int)grow.size(), 64, 0, s>>>((int)grow.size(), drows, doff, dts, xv, yv, scr, cnt, ovf);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(s));
        HIPC(hipMemsetAsync(ovf, 0, sizeof(int32_t), s));
        rowptr_and_bins();
    }
    if (nnz > INT32_MAX) fail(CAMG_E_NOMEM, "sparse product has more than 2^31-1 nonzeros");
    Z.nnz = nnz;
    Z.ci = out.alloc<int32_t>(padded(nnz));
    Z.v = out.alloc<double>(padded(nnz));

    // 4. fill
    if (thrp >= 0)
        k_thread_rows<true><<<nblk(nr, 256), 256, 0, s>>>(nr, xv, yv, prod, thrp, nullptr, Z.rp, Z.ci, Z.v);
    HIPC(hipGetLastError());
    launch_fill<128, 64, kWPB>(hb[0], brows2 + 0 * (size_t)nr, xv, yv, Z.rp, Z.ci, Z.v, s);
    launch_fill<512, 256, kWPB>(hb[1], brows2 + 1 * (size_t)nr, xv, yv, Z.rp, Z.ci, Z.v, s);
    launch_fill<2048, 1024, kWPB>(hb[2], brows2 + 2 * (size_t)nr, xv, yv, Z.rp, Z.ci, Z.v, s);
    launch_fill<8192, 4096, 1>(hb[3], brows2 + 3 * (size_t)nr, xv, yv, Z.rp, Z.ci, Z.v, s);
    if (hb[4] > 0) {
        std::vector<int32_t> rows(hb[4]);
        std::vector<int32_t> zrp(nr + 1);
        HIPC(hipMemcpy(rows.data(), brows2 + 4 * (size_t)nr, sizeof(int32_t) * rows.size(), hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(zrp.data(), Z.rp, sizeof(int32_t) * (nr + 1), hipMemcpyDeviceToHost));
        std::vector<int32_t> gts;
        std::vector<int64_t> gio, gdo;
        int64_t itot = 0, dtot = 0;
        for (int r : rows) {
            const int u = zrp[r + 1] - zrp[r];
            const int ts = next_pow2(2 * (int64_t)u + 1);
            const int np = next_pow2(u);
            gts.push_back(ts);
            gio.push_back(itot);
            gdo.push_back(dtot);
            itot += 2 * (int64_t)ts + np;
            dtot += u;
        }
        Pool g(s);
        const int m = (int)rows.size();
        int *iscr = g.alloc<int>((size_t)itot);
        double *dscr = g.alloc<double>((size_t)std::max<int64_t>(dtot, 1));
        int32_t *drows = g.alloc<int32_t>(m);
        int32_t *dts = g.alloc<int32_t>(m);
        int64_t *dio = g.alloc<int64_t>(m);
        int64_t *ddo = g.alloc<int64_t>(m);
        int *ctr = g.alloc<int>(m);
        HIPC(hipMemcpyAsync(drows, rows.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(dts, gts.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(dio, gio.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(ddo, gdo.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s));
        k_fill_glb<<<m, 64, 0, s>>>(m, drows, dio, ddo, dts, xv, yv, Z.rp, Z.ci, Z.v, iscr, dscr, ctr);
        HIPC(hipGetLastError());
        HIPC(hipStreamSynchronize(s));
    }
}

// A_c = R (A P) (eq. AcDef).  When the products of A P exceed `chunk`, the
// coarse rows are taken in consecutive chunks: a chunk needs the rows of
// A P between the smallest and the largest fine index its rows of R touch,
// which are formed from the same rows of A; the chunk's rows of A_c are then
// R_chunk times that window.  Every entry receives the same products in the
// same order as in the unchunked product, so the result is bitwise the same;
// only the temporary memory shrinks.
void galerkin(const Csr &A, const Csr &P, const Csr &R, Csr &Ac, int64_t chunk, Pool &out, Pool &tmp,
              hipStream_t s) {
    const int64_t budget = chunk > 0 ? chunk : (int64_t)1 << 30;
    const int nf = A.nr, ncr = R.nr;
    int64_t *prod = tmp.alloc<int64_t>(std::max(nf, 1));
    int64_t *pref = tmp.alloc<int64_t>((size_t)nf + 1);
    CsrView av{A.rp, A.ci, A.v}, pv{P.rp, P.ci, P.v};
    row_products(nf, A.nnz, av, pv, prod, s);
    scan_i64(prod, pref, nf, tmp, s);
    int64_t total = 0;
    HIPC(hipMemcpyAsync(&total, pref + nf, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (total <= budget || ncr <= 1) {
        Csr AP;
        spgemm(A, P, AP, tmp, tmp, s);
        spgemm(R, AP, Ac, out, tmp, s);
        return;
    }
    // plan the chunks on the host
    std::vector<int64_t> hpref((size_t)nf + 1);
    std::vector<int32_t> lo(ncr), hi(ncr), rrp((size_t)ncr + 1);
    {
        int32_t *dlo = tmp.alloc<int32_t>(ncr), *dhi = tmp.alloc<int32_t>(ncr);
        k_row_span<<<nblk(ncr, kBlock), kBlock, 0, s>>>(ncr, R.rp, R.ci, dlo, dhi);
        HIPC(hipGetLastError());
        HIPC(hipMemcpyAsync(hpref.data(), pref, sizeof(int64_t) * hpref.size(), hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(lo.data(), dlo, sizeof(int32_t) * ncr, hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(hi.data(), dhi, sizeof(int32_t) * ncr, hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(rrp.data(), R.rp, sizeof(int32_t) * rrp.size(), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
    }
    struct Part {
        int c0, c1, f0, f1;
        Csr C;
    };
    std::vector<Part> parts;
    for (int c0 = 0; c0 < ncr;) {
        int f0 = lo[c0], f1 = hi[c0], c1 = c0 + 1;
        while (c1 < ncr) {
            const int a = std::min(f0, lo[c1]), b = std::max(f1, hi[c1]);
            if (a <= b && hpref[b + 1] - hpref[a] > budget) break;
            f0 = a;
            f1 = b;
            ++c1;
        }
        if (f0 > f1) f0 = f1 = 0;  // rows of R without entries
        parts.push_back({c0, c1, f0, f1, Csr{}});
        c0 = c1;
    }
    Pool keep(s);
    int64_t nnz = 0;
    for (Part &pt : parts) {
        Pool g(s);
        Csr Aw;  // rows f0..f1 of A (row pointers index A's arrays)
        Aw.nr = pt.f1 - pt.f0 + 1;
        Aw.nc = A.nc;
        Aw.rp = A.rp + pt.f0;
        Aw.ci = A.ci;
        Aw.v = A.v;
        Csr APw;
        spgemm(Aw, P, APw, g, g, s);
        const int m = pt.c1 - pt.c0;
        const int64_t e0 = rrp[pt.c0], ne = (int64_t)rrp[pt.c1] - e0;
        Csr Rc;
        Rc.nr = m;
        Rc.nc = Aw.nr;
        Rc.nnz = ne;
        Rc.rp = g.alloc<int32_t>((size_t)m + 1);
        Rc.ci = g.alloc<int32_t>(padded(std::max<int64_t>(ne, 1)));
        Rc.v = R.v + e0;
        k_slice_rows<<<nblk(m + 1, kBlock), kBlock, 0, s>>>(m, R.rp, pt.c0, Rc.rp);
        if (ne > 0) k_shift_cols<<<nblk(ne, kBlock), kBlock, 0, s>>>(ne, R.ci + e0, pt.f0, Rc.ci);
        HIPC(hipGetLastError());
        spgemm(Rc, APw, pt.C, keep, g, s);
        HIPC(hipStreamSynchronize(s));
        nnz += pt.C.nnz;
    }
    if (nnz > INT32_MAX) fail(CAMG_E_NOMEM, "Galerkin product has more than 2^31-1 nonzeros");
    Ac.nr = ncr;
    Ac.nc = P.nc;
    Ac.nnz = nnz;
    Ac.rp = out.alloc<int32_t>((size_t)ncr + 1);
    Ac.ci = out.alloc<int32_t>(padded(nnz));
    Ac.v = out.alloc<double>(padded(nnz));
    int64_t base = 0;
    for (const Part &pt : parts) {
        const int m = pt.c1 - pt.c0;
        k_offset_rp<<<nblk(m + 1, kBlock), kBlock, 0, s>>>(m, pt.C.rp, base, Ac.rp + pt.c0);
        HIPC(hipGetLastError());
        if (pt.C.nnz > 0) {
            HIPC(hipMemcpyAsync(Ac.ci + base, pt.C.ci, sizeof(int32_t) * pt.C.nnz, hipMemcpyDeviceToDevice, s));
            HIPC(hipMemcpyAsync(Ac.v + base, pt.C.v, sizeof(double) * pt.C.nnz, hipMemcpyDeviceToDevice, s));
        }
        base += pt.C.nnz;
    }
    HIPC(hipStreamSynchronize(s));
}

}  // namespace camg
