// Hierarchy set-up kernels (Alg. "AMG Set-up" of the paper): input checks,
// strength of connection, PMIS rounds, interpolation, transpose,
// Jacobi weights and the dense last-level factorisation.
//
// Every kernel that produces a value the CPU reference also produces does
// the same floating-point operations in the same order (sums in CSR order,
// no fused multiply-add: the library is built with -ffp-contract=off), so
// patterns and values of the hierarchy are reproducible bit for bit.
#include "devutil.hpp"
#include "internal.hpp"

namespace camg {

namespace {

inline int nblocks(int64_t n, int bs = kBlock) { return (int)((n + bs - 1) / bs); }

// wavefront-scope barrier: LDS writes of the wavefront are visible to all its lanes
#define FSAI_SYNC()                                             \
    do {                                                        \
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                        \
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
    } while (0)


// ---------------------------------------------------------------- scan
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

template <class T>
__device__ void block_exclusive_scan(int64_t (&v)[kScanItems], int64_t &total) {
    int64_t local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t t = v[i];
        v[i] = local;
        local += t;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __shared__ int64_t ws[kBlock / 64];
    if (lane == 63) ws[w] = x;
    __syncthreads();
    int64_t base = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        if (i < w) base += ws[i];
        total += ws[i];
    }
    const int64_t excl = base + x - local;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) v[i] += excl;
    __syncthreads();
}

// Block results folded into one device word: the maximum only by a block
// whose value exceeds what the word holds already (values only grow, so a
// stale read costs an atomic at most), and "some point left" by the first
// blocks that find the word at zero.  Either keeps the result exact while
// most of the grid's blocks skip the atomic (one atomic per block on one
// address serialises the grid).
__device__ __forceinline__ void fold_max(unsigned long long *w, unsigned long long v) {
    if (v > __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(w, v);
}
__device__ __forceinline__ void fold_max(int32_t *w, int32_t v) {
    if (v > __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(w, v);
}
__device__ __forceinline__ void fold_any(int32_t *w, int32_t v) {
    if (v > 0 && __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) atomicAdd(w, v);
}

template <class T>
__global__ void k_scan_tiles(const T *in, int n, int64_t *tile_sum) {
    int64_t v[kScanItems];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < n) ? (int64_t)in[base + i] : 0;
    int64_t total;
    block_exclusive_scan<T>(v, total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// single block: exclusive scan of the tile sums in place, total in [nt]
__global__ void k_scan_tile_sums(int64_t *ts, int nt) {
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nt; b0 += kScanTile) {
        int64_t v[kScanItems];
        const int base = b0 + threadIdx.x * kScanItems;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < nt) ? ts[base + i] : 0;
        int64_t total;
        block_exclusive_scan<int64_t>(v, total);
        const int64_t c = carry;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i)
            if (base + i < nt) ts[base + i] = v[i] + c;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + total;
        __syncthreads();
    }
    if (threadIdx.x == 0) ts[nt] = carry;
}

template <class T>
__global__ void k_scan_apply(const T *in, int n, const int64_t *ts, int64_t *out) {
    int64_t v[kScanItems];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < n) ? (int64_t)in[base + i] : 0;
    int64_t total;
    block_exclusive_scan<T>(v, total);
    const int64_t off = ts[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) out[base + i] = v[i] + off;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = ts[gridDim.x];
}

template <class T>
void scan_impl(const T *in, int64_t *out, int n, Pool &tmp, hipStream_t s) {
    const int nt = std::max(1, (n + kScanTile - 1) / kScanTile);
    int64_t *ts = tmp.alloc<int64_t>(nt + 1);
    k_scan_tiles<T><<<nt, kBlock, 0, s>>>(in, n, ts);
    k_scan_tile_sums<<<1, kBlock, 0, s>>>(ts, nt);
    k_scan_apply<T><<<nt, kBlock, 0, s>>>(in, n, ts, out);
    HIPC(hipGetLastError());
}

__global__ void k_narrow(const int64_t *v, int32_t *o, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) o[i] = (int32_t)v[i];
}

// ---------------------------------------------------------------- validation
__global__ void k_val_rowptr(int n, int64_t nnz, const int32_t *rp, int32_t *flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) atomicOr(&flags[0], 1);
    if (i < n && rp[i + 1] < rp[i]) atomicOr(&flags[0], 1);
}

// ---- per-row set-up work with G lanes per row (G a power of two <= 64):
// lane sl of a row's group takes the row's entries sl, sl + G, ..., so the
// group's loads are coalesced.  Whole groups run every loop and shuffle
// (rows past n have empty bounds).  Maxima, integer counts and per-entry
// values do not depend on the order of the lanes, and the one ordered sum
// (Gershgorin) is formed in CSR order, so every result is the one a single
// thread walking the row would give.
template <int G>
__device__ __forceinline__ int group_row(int n, int &sl) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    sl = (int)(t & (G - 1));
    return (int)(t / G);
}

// Column range and order, finite values, a positive diagonal, and the
// largest |a_ij| (for the symmetry tolerance), checked with G lanes per row.
template <int G>
__global__ void __launch_bounds__(kBlock) k_val_rows_g(int n, const int32_t *rp, const int32_t *ci, const double *v,
                                                       int32_t *flags, unsigned long long *amax) {
    int sl;
    const int i = group_row<G>(n, sl);
    const int e0 = i < n ? rp[i] : 0, e1 = i < n ? rp[i + 1] : 0;
    int bad_col = 0, bad_val = 0, diag = 0, bad_diag = 0;
    double m = 0.0;
    for (int e = e0 + sl; e < e1; e += G) {
        const int c = ci[e];
        if (c < 0 || c >= n || (e > e0 && c <= ci[e - 1])) bad_col = 1;
        const double a = v[e];
        if (!isfinite(a)) bad_val = 1;
        else if (fabs(a) > m) m = fabs(a);
        if (c == i) {
            diag = 1;
            if (!(a > 0.0)) bad_diag = 1;
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) diag |= __shfl_xor(diag, o, G);
    if (bad_col) atomicOr(&flags[1], 1);
    if (bad_val) atomicOr(&flags[2], 1);
    if (i < n && sl == 0 && !diag) atomicOr(&flags[3], 1);
    if (bad_diag) atomicOr(&flags[5], 1);
    const unsigned long long bm = block_max_u64<kBlock>((unsigned long long)__double_as_longlong(m));
    if (threadIdx.x == 0) fold_max(amax, bm);
}

// tpos[e] = position of entry (j, i) in row j for entry e = (i, j); checks
// structural and numerical symmetry when flags != nullptr.
template <int G>
__global__ void __launch_bounds__(kBlock) k_tpos_g(int n, const int32_t *rp, const int32_t *ci, const double *v,
                                                   const unsigned long long *amax, int32_t *flags, int32_t *tpos) {
    int sl;
    const int i = group_row<G>(n, sl);
    if (i >= n) return;  // no shuffles below
    const double tol = flags ? 1e-12 * __longlong_as_double((long long)*amax) : 0.0;
    int bad = 0;
    for (int e = rp[i] + sl; e < rp[i + 1]; e += G) {
        const int j = ci[e];
        const int t = find_col(ci, rp[j], rp[j + 1], i);
        tpos[e] = t;
        if (t < 0) bad = 1;
        else if (flags && fabs(v[e] - v[t]) > tol) bad = 1;
    }
    if (bad && flags) atomicOr(&flags[4], 1);
}

// ---------------------------------------------------------------- strength
// Classical strength with threshold: m_i = max_{k != i} (-a_ik);
// j in S_i iff j != i, m_i > 0 and -a_ij >= theta * m_i (one rounded product).
template <int G>
__global__ void __launch_bounds__(kBlock) k_strength_g(int n, const int32_t *rp, const int32_t *ci, const double *v,
                                                       double theta, uint8_t *strong) {
    int sl;
    const int i = group_row<G>(n, sl);
    const int e0 = i < n ? rp[i] : 0, e1 = i < n ? rp[i + 1] : 0;
    int have = 0;
    double m = 0.0;
    for (int e = e0 + sl; e < e1; e += G) {
        if (ci[e] == i) continue;
        const double neg = -v[e];
        if (!have || neg > m) {
            m = neg;
            have = 1;
        }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {  // the group's maximum (and whether it has any entry)
        const int oh = __shfl_xor(have, o, G);
        const double om = __shfl_xor(m, o, G);
        if (oh && (!have || om > m)) {
            m = om;
            have = 1;
        }
    }
    const double thr = theta * m;
    for (int e = e0 + sl; e < e1; e += G) {
        const int j = ci[e];
        strong[e] = (j != i && have && m > 0.0 && -v[e] >= thr) ? 1 : 0;
    }
}

// |S_i^T| = number of rows j with i in S_j = sum over row i of the strong
// flags at the transposed positions (the pattern is symmetric)
template <int G>
__global__ void __launch_bounds__(kBlock) k_stcount_g(int n, const int32_t *rp, const int32_t *tpos,
                                                      const uint8_t *strong, int32_t *stcnt) {
    int sl;
    const int i = group_row<G>(n, sl);
    const int e0 = i < n ? rp[i] : 0, e1 = i < n ? rp[i + 1] : 0;
    int c = 0;
    for (int e = e0 + sl; e < e1; e += G) c += strong[tpos[e]];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, G);
    if (i < n && sl == 0) stcnt[i] = c;
}

// Jacobi weight: dinv_i = 1 / a_ii and q_i = (sum_j |a_ij|) / a_ii (CSR
// order); the max of q over rows is the Gershgorin bound of rho(D^{-1} A).
// The group reads the row G entries at a time and every lane adds them up
// one by one in CSR order from lane 0 to lane G-1 of each chunk, so s_i is
// the sequential sum.
template <int G>
__global__ void __launch_bounds__(kBlock) k_diag_gersh_g(int n, const int32_t *rp, const int32_t *ci,
                                                         const double *v, double *dinv, unsigned long long *qmax,
                                                         int32_t *flags) {
    int sl;
    const int i = group_row<G>(n, sl);
    const int e0 = i < n ? rp[i] : 0, e1 = i < n ? rp[i + 1] : 0;
    double s = 0.0, d = 0.0;
    int hd = 0;
    for (int c = e0; c < e1; c += G) {
        const int e = c + sl;
        double a = 0.0;
        if (e < e1) {
            a = fabs(v[e]);
            if (ci[e] == i) {
                d = v[e];
                hd = 1;
            }
        }
        const int cnt = min(G, e1 - c);
        for (int k = 0; k < cnt; ++k) s = s + __shfl(a, k, G);
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {  // the diagonal from the lane that read it
        const int oh = __shfl_xor(hd, o, G);
        const double od = __shfl_xor(d, o, G);
        if (oh) {
            d = od;
            hd = 1;
        }
    }
    double q = 0.0;
    if (i < n && sl == 0) {
        if (!(d > 0.0)) {
            atomicOr(&flags[5], 1);
            dinv[i] = 0.0;
        } else {
            dinv[i] = 1.0 / d;
            q = s / d;
        }
    }
    const unsigned long long bm = block_max_u64<kBlock>((unsigned long long)__double_as_longlong(q));
    if (threadIdx.x == 0) fold_max(qmax, bm);
}

// awd_e = a_e * wd_{col e}, one thread per nonzero
__global__ void k_scale_entries(int64_t nnz, const int32_t *ci, const double *v, const double *wd, double *awd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) awd[e] = v[e] * wd[ci[e]];
}

// lanes per row for the group kernels: the smallest power of two covering
// the mean row length, at most 64
inline int group_lanes(int n, int64_t nnz) {
    const double mean = n > 0 ? (double)nnz / n : 1.0;
    int g = 1;
    while (g < 64 && g < mean) g <<= 1;
    return g;
}
inline int group_blocks(int n, int g) { return (int)(((int64_t)n * g + kBlock - 1) / kBlock); }
constexpr int kOrderedLanes = 8;  // most lanes per row of a group kernel with an ordered sum

#define CAMG_G_SWITCH(g, ...)                              \
    switch (g) {                                           \
    case 1: { constexpr int G = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int G = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int G = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int G = 8; __VA_ARGS__; } break;   \
    case 16: { constexpr int G = 16; __VA_ARGS__; } break; \
    case 32: { constexpr int G = 32; __VA_ARGS__; } break; \
    default: { constexpr int G = 64; __VA_ARGS__; } break; \
    }

// ---------------------------------------------------------------- PMIS
constexpr int8_t kF = -1, kU = 0, kC = 1;

__global__ void k_pmis_init(int n, const int32_t *stcnt, uint64_t seed, int level, uint64_t *u, int8_t *state,
                            int32_t *undecided) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int und = 0;
    if (i < n) {
        const uint64_t c = ((uint64_t)(uint32_t)level << 40) + (uint64_t)(uint32_t)i;
        u[i] = splitmix64(seed, c) >> 11;
        const int8_t s = stcnt[i] == 0 ? kF : kU;
        state[i] = s;
        und = (s == kU);
    }
    const long long bu = block_sum_ll<kBlock>(und);
    if (threadIdx.x == 0) fold_any(undecided, (int32_t)bu);
}

__device__ __forceinline__ bool key_gt(const int32_t *cnt, const uint64_t *u, int a, int b) {
    const int ca = cnt[a], cb = cnt[b];
    if (ca != cb) return ca > cb;
    const uint64_t ua = u[a], ub = u[b];
    if (ua != ub) return ua > ub;
    return a > b;
}

// ---------------------------------------------------------------- PMIS rounds, G lanes per row
// Selection: undecided i joins the new C set if its measure beats every
// undecided neighbour in S_i u S_i^T (state as at the start of the round).
// Whether some neighbour beats i does not depend on the order it is found in.
template <int G>
__global__ void __launch_bounds__(kBlock) k_pmis_select_g(int n, const int32_t *rp, const int32_t *ci,
                                                          const uint8_t *strong, const int32_t *tpos,
                                                          const int32_t *stcnt, const uint64_t *u,
                                                          const int8_t *state, int8_t *newc) {
    int sl;
    const int i = group_row<G>(n, sl);
    const bool und = i < n && state[i] == kU;
    const int e0 = und ? rp[i] : 0, e1 = und ? rp[i + 1] : 0;
    int beaten = 0;
    for (int e = e0 + sl; e < e1 && !beaten; e += G) {
        const int j = ci[e];
        if (j == i || state[j] != kU) continue;
        const int te = tpos[e];
        if (!(strong[e] || (te >= 0 && strong[te]))) continue;
        if (key_gt(stcnt, u, j, i)) beaten = 1;
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) beaten |= __shfl_xor(beaten, o, G);
    if (i < n && sl == 0) newc[i] = (und && !beaten) ? 1 : 0;
}

// Update: new C points become C; undecided points that depend strongly on
// a new C point become F.
template <int G>
__global__ void __launch_bounds__(kBlock) k_pmis_update_g(int n, const int32_t *rp, const int32_t *ci,
                                                          const uint8_t *strong, const int8_t *newc, int8_t *state,
                                                          int32_t *undecided) {
    int sl;
    const int i = group_row<G>(n, sl);
    const bool und = i < n && state[i] == kU;
    const bool look = und && !newc[i];
    const int e0 = look ? rp[i] : 0, e1 = look ? rp[i + 1] : 0;
    int f = 0;
    for (int e = e0 + sl; e < e1 && !f; e += G)
        if (strong[e] && newc[ci[e]]) f = 1;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) f |= __shfl_xor(f, o, G);
    int left = 0;
    if (und && sl == 0) {
        if (newc[i]) state[i] = kC;
        else if (f) state[i] = kF;
        else left = 1;
    }
    const long long bu = block_sum_ll<kBlock>(left);
    if (threadIdx.x == 0) fold_any(undecided, (int32_t)bu);
}

// ---------------------------------------------------------------- direct interpolation, G lanes per row
template <int G>
__global__ void __launch_bounds__(kBlock) k_interp_count_g(int n, const int32_t *rp, const int32_t *ci,
                                                           const uint8_t *strong, const int8_t *cf, int32_t *cnt) {
    int sl;
    const int i = group_row<G>(n, sl);
    const bool frow = i < n && cf[i] != kC;
    const int e0 = frow ? rp[i] : 0, e1 = frow ? rp[i + 1] : 0;
    int c = 0;
    for (int e = e0 + sl; e < e1; e += G)
        if (strong[e] && cf[ci[e]] == kC) ++c;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, G);
    if (i < n && sl == 0) cnt[i] = frow ? c : 1;
}

// C row: a single 1 at cmap(i).  F row: w_ij = -(alpha_i a_ij) / d_i over
// C_i^S, d_i = a_ii + positive off-diagonals, alpha_i = (sum of negative
// off-diagonals) / (sum over C_i^S of a_ij).  The lanes read G entries at a
// time; every lane then adds the G terms in CSR order, so each of the three
// sums is the chain a single thread walking the row would form, and the
// weights go out in CSR order at ranks taken from a ballot.
template <int G>
__global__ void __launch_bounds__(kBlock) k_interp_fill_g(int n, const int32_t *rp, const int32_t *ci,
                                                          const double *v, const uint8_t *strong, const int8_t *cf,
                                                          const int64_t *cmap, const int32_t *prp, int32_t *pci,
                                                          double *pv) {
    int sl;
    const int i = group_row<G>(n, sl);
    const bool isc = i < n && cf[i] == kC;
    int o = i < n ? prp[i] : 0;
    if (isc && sl == 0) {
        pci[o] = (int32_t)cmap[i];
        pv[o] = 1.0;
    }
    const bool frow = i < n && !isc && prp[i + 1] != o;
    const int e0 = frow ? rp[i] : 0, e1 = frow ? rp[i + 1] : 0;
    double d = 0.0;
    int hd = 0;
    for (int e = e0 + sl; e < e1; e += G)
        if (ci[e] == i) {
            d = v[e];
            hd = 1;
        }
#pragma unroll
    for (int q = G / 2; q > 0; q >>= 1) {  // the diagonal from the lane that read it
        const int oh = __shfl_xor(hd, q, G);
        const double od = __shfl_xor(d, q, G);
        if (oh) {
            d = od;
            hd = 1;
        }
    }
    double num = 0.0, den = 0.0;
    for (int c = e0; c < e1; c += G) {
        const int e = c + sl;
        double a = 0.0;
        int kind = 0;  // bit 0: positive off-diagonal, bit 1: negative off-diagonal, bit 2: in C_i^S
        if (e < e1) {
            const int j = ci[e];
            a = v[e];
            if (j != i) kind = a > 0.0 ? 1 : (a < 0.0 ? 2 : 0);
            if (strong[e] && cf[j] == kC) kind |= 4;
        }
        const int cnt = min(G, e1 - c);
        for (int k = 0; k < cnt; ++k) {
            const double ak = __shfl(a, k, G);
            const int kk = __shfl(kind, k, G);
            if (kk & 1) d = d + ak;
            else if (kk & 2) num = num + ak;
            if (kk & 4) den = den + ak;
        }
    }
    const double alpha = num / den;
    const int gbase = (int)(threadIdx.x & 63) & ~(G - 1);
    const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
    for (int c = e0; c < e1; c += G) {
        const int e = c + sl;
        int j = 0, sc = 0;
        if (e < e1) {
            j = ci[e];
            sc = strong[e] && cf[j] == kC;
        }
        const unsigned long long g = (__ballot(sc) >> gbase) & gmask;
        if (sc) {
            const int r = o + __popcll(g & ((1ull << sl) - 1));
            pci[r] = (int32_t)cmap[j];
            pv[r] = -(alpha * v[e]) / d;
        }
        o += __popcll(g);
    }
}

__global__ void k_cf_flags(int n, const int8_t *cf, int32_t *isc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) isc[i] = cf[i] == kC ? 1 : 0;
}

// ---------------------------------------------------------------- direct interpolation
// ---------------------------------------------------------------- transpose
__global__ void k_col_count(int64_t nnz, const int32_t *ci, int32_t *cnt) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[ci[e]], 1);
}

__global__ void k_transpose_fill(int nr, const int32_t *rp, const int32_t *ci, const double *v, int32_t *fill,
                                 int32_t *tci, double *tv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int c = ci[e];
        const int pos = atomicAdd(&fill[c], 1);
        tci[pos] = i;
        tv[pos] = v[e];
    }
}

// rows of the transpose come out of k_transpose_fill in arbitrary order and
// are sorted by column: rows of at most `smax` entries by one thread
// (insertion sort), rows of at most kSortWave by a wavefront, longer ones by
// a workgroup (k_sort_rows_block); the longer two rank the entries.  smax
// is kSortShort when the transpose has at least kSortThreadRows rows, else
// 1: a thread's sort is a chain of dependent loads, hidden only when many
// rows run at once.
constexpr int kSortShort = 32, kSortWave = 1024, kSortBlockLds = 8192, kSortThreadRows = 131072;

__global__ void k_sort_rows(int nr, const int32_t *rp, int32_t *ci, double *v, int smax) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    const int e0 = rp[i], e1 = rp[i + 1];
    if (e1 - e0 > smax) return;
    for (int e = e0 + 1; e < e1; ++e) {
        const int c = ci[e];
        const double x = v[e];
        int f = e - 1;
        while (f >= e0 && ci[f] > c) {
            ci[f + 1] = ci[f];
            v[f + 1] = v[f];
            --f;
        }
        ci[f + 1] = c;
        v[f + 1] = x;
    }
}

// one wavefront per row of smax < length <= kSortWave entries: the
// row is staged in LDS and every entry moves to its rank (the columns of a
// row are distinct)
__global__ void __launch_bounds__(256) k_sort_rows_wave(int nr, const int32_t *rp, int32_t *ci, double *v, int smax) {
    __shared__ int kc[4][kSortWave];
    __shared__ double kv[4][kSortWave];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int i = blockIdx.x * 4 + w;
    if (i >= nr) return;
    const int e0 = rp[i], L = rp[i + 1] - e0;
    if (L <= smax || L > kSortWave) return;
    for (int t = lane; t < L; t += kWave) {
        kc[w][t] = ci[e0 + t];
        kv[w][t] = v[e0 + t];
    }
    FSAI_SYNC();
    for (int t = lane; t < L; t += kWave) {
        const int c = kc[w][t];
        int r = 0;
        for (int u = 0; u < L; ++u) r += kc[w][u] < c ? 1 : 0;
        ci[e0 + r] = c;
        v[e0 + r] = kv[w][t];
    }
}

// indices of the rows longer than minlen (in any order) and their number
__global__ void k_long_rows(int nr, const int32_t *rp, int minlen, int32_t *list, int32_t *count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr && rp[i + 1] - rp[i] > minlen) list[atomicAdd(count, 1)] = i;
}

// one workgroup per listed row: the unsorted row is read from a copy (sci,
// sv) and every entry is written at its rank; the keys are staged in LDS
// when they fit
__global__ void __launch_bounds__(1024) k_sort_rows_block(const int32_t *list, const int32_t *rp,
                                                          const int32_t *sci, const double *sv, int32_t *ci,
                                                          double *v) {
    __shared__ int kc[kSortBlockLds];
    const int i = list[blockIdx.x];
    const int e0 = rp[i], L = rp[i + 1] - e0;
    const bool lds = L <= kSortBlockLds;
    if (lds) {
        for (int t = threadIdx.x; t < L; t += blockDim.x) kc[t] = sci[e0 + t];
        __syncthreads();
    }
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const int c = sci[e0 + t];
        int r = 0;
        if (lds) {
            for (int u = 0; u < L; ++u) r += kc[u] < c ? 1 : 0;
        } else {
            for (int u = 0; u < L; ++u) r += sci[e0 + u] < c ? 1 : 0;
        }
        ci[e0 + r] = c;
        v[e0 + r] = sv[e0 + t];
    }
}

// ---------------------------------------------------------------- Jacobi weight
__global__ void k_scale(int n, double omega, const double *dinv, double *wd) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wd[i] = omega * dinv[i];
}

__global__ void k_to_f32(int64_t n, const double *in, float *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

// ---------------------------------------------------------------- last level
__global__ void k_dense_zero(int64_t nn, double *D) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nn) D[i] = 0.0;
}

__global__ void k_dense_from_csr(int n, const int32_t *rp, const int32_t *ci, const double *v, double *D) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) D[(int64_t)i * n + ci[e]] = v[e];
}

// Right-looking dense Cholesky by one block, in place (lower triangle).
__global__ void __launch_bounds__(1024) k_cholesky(int n, double *D, int32_t *flags) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (threadIdx.x == 0) {
            const double s = D[(int64_t)j * n + j];
            if (!(s > 0.0)) bad = 1;
            else D[(int64_t)j * n + j] = sqrt(s);
        }
        __syncthreads();
        if (bad) break;
        const double ljj = D[(int64_t)j * n + j];
        for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) D[(int64_t)i * n + j] = D[(int64_t)i * n + j] / ljj;
        __syncthreads();
        // trailing update of the lower triangle: rows i > j, columns j < k <= i
        // (one wavefront per row, lanes over the row's columns)
        const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
        for (int i = j + 1 + wave; i < n; i += nw) {
            const double lij = D[(int64_t)i * n + j];
            for (int k = j + 1 + lane; k <= i; k += 64)
                D[(int64_t)i * n + k] = D[(int64_t)i * n + k] - lij * D[(int64_t)k * n + j];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && bad) atomicOr(&flags[5], 1);
}

// Blocked right-looking Cholesky for n <= kCholMfmaMax by one 512-thread
// workgroup, in place (lower triangle).  Per 16-column panel: the diagonal
// block is factorised in LDS (one barrier per column; two copies alternate,
// so a step reads one while writing the other; padding beyond n is the
// identity), the rows below solve against it (a thread per row), and the
// trailing lower triangle is updated tile by tile on the matrix cores:
// A_IJ -= L_I L_J^T over the panel's 16 columns with v_mfma_f64_16x16x4f64,
// one wavefront per 16x16 tile (lane l supplies row/column l%16 at inner
// index l/16 and receives rows l/16 + 4r of column l%16).
constexpr int kCholMfmaMax = 256;
typedef double chol_d4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(512) k_cholesky_mfma(int n, double *D, int32_t *flags) {
    __shared__ double Lb[2][16][17];
    __shared__ int bad;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    if (tid == 0) bad = 0;
    __syncthreads();
    const int np = (n + 15) / 16;
    for (int p = 0; p < np; ++p) {
        const int c0 = 16 * p, cw = min(16, n - c0);
        if (tid < 256) {
            const int r = tid / 16, q = tid % 16;
            Lb[0][r][q] = (r < cw && q < cw) ? D[(size_t)(c0 + r) * n + c0 + q] : (r == q ? 1.0 : 0.0);
        }
        __syncthreads();
        for (int c = 0; c < 16; ++c) {
            const int cur = c & 1, nxt = cur ^ 1;
            if (tid < 256) {
                const int r = tid / 16, q = tid % 16;
                double out = Lb[cur][r][q];
                if (q >= c && q <= r) {
                    const double d = Lb[cur][c][c];
                    if (r == c && q == c && !(d > 0.0)) bad = 1;
                    const double piv = sqrt(d);
                    if (q == c) out = r == c ? piv : Lb[cur][r][c] / piv;
                    else out = Lb[cur][r][q] - (Lb[cur][r][c] / piv) * (Lb[cur][q][c] / piv);
                }
                Lb[nxt][r][q] = out;
            }
            __syncthreads();
        }
        // 16 steps: the factor is back in copy 0
        if (tid < 256) {
            const int r = tid / 16, q = tid % 16;
            if (r < cw && q <= r) D[(size_t)(c0 + r) * n + c0 + q] = Lb[0][r][q];
        }
        // rows below the block: x L11^T = a, column by column, in place
        for (int i = c0 + 16 + tid; i < n; i += 512) {
            double *x = D + (size_t)i * n + c0;
            for (int c = 0; c < 16; ++c) {
                double t = x[c];
                for (int q = 0; q < c; ++q) t = t - x[q] * Lb[0][c][q];
                x[c] = t / Lb[0][c][c];
            }
        }
        __syncthreads();
        // trailing update of the tiles (I, J), p < J <= I < np
        const int side = np - p - 1;
        const int ntile = side * (side + 1) / 2;
        const int li = lane % 16, lk = lane / 16;
        for (int t = wave; t < ntile; t += 8) {
            int I = 0, tt = t;
            while (tt > I) {
                tt -= I + 1;
                ++I;
            }
            const int i0 = 16 * (p + 1 + I), j0 = 16 * (p + 1 + tt);
            chol_d4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + lk + 4 * r, j = j0 + li;
                acc[r] = (i < n && j < n) ? D[(size_t)i * n + j] : 0.0;
            }
            const int ia = i0 + li, jb = j0 + li;
#pragma unroll
            for (int k0 = 0; k0 < 16; k0 += 4) {
                const int k = c0 + k0 + lk;
                const double a = ia < n ? -D[(size_t)ia * n + k] : 0.0;
                const double b = jb < n ? D[(size_t)jb * n + k] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + lk + 4 * r, j = j0 + li;
                if (i < n && j <= i) D[(size_t)i * n + j] = acc[r];
            }
        }
        __syncthreads();
    }
    if (tid == 0 && bad) atomicOr(&flags[5], 1);
}

// X = (L L^T)^{-1}: one wavefront per column j, whose vector lives in LDS.
// Forward L y = e_j row by row from row j (y is zero above it), the inner
// products split over the lanes; backward L^T x = y from the last row up,
// each x_i then taken out of the rows above it with row i of L.  Both sweeps
// read rows of L (contiguous), the next row's first kInvAhead * 64 entries
// loaded while the current row is used, so a step waits for LDS and the
// wavefront barrier rather than for memory.
constexpr int kInvAhead = 4;
__global__ void __launch_bounds__(64) k_chol_inverse(int n, const double *L, double *X) {
    extern __shared__ double y[];  // n doubles
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    if (j >= n) return;
    for (int k = lane; k < n; k += 64) y[k] = 0.0;
    double cur[kInvAhead], nxt[kInvAhead];
    // forward: entries k in [j, i) of row i
    auto fwd_row = [&](int i, double *r) {
#pragma unroll
        for (int m = 0; m < kInvAhead; ++m) {
            const int k = j + lane + 64 * m;
            r[m] = (i < n && k < i) ? L[(int64_t)i * n + k] : 0.0;
        }
    };
    fwd_row(j, cur);
    double dcur = L[(int64_t)j * n + j];
    __syncthreads();
    for (int i = j; i < n; ++i) {
        fwd_row(i + 1, nxt);
        const double dnxt = i + 1 < n ? L[(int64_t)(i + 1) * n + i + 1] : 1.0;
        double t = 0.0;
#pragma unroll
        for (int m = 0; m < kInvAhead; ++m) {
            const int k = j + lane + 64 * m;
            if (k < i) t += cur[m] * y[k];
        }
        for (int k = j + lane + 64 * kInvAhead; k < i; k += 64) t += L[(int64_t)i * n + k] * y[k];
        t = wave_sum(t);
        if (lane == 0) y[i] = ((i == j ? 1.0 : 0.0) - t) / dcur;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kInvAhead; ++m) cur[m] = nxt[m];
        dcur = dnxt;
    }
    // backward: entries k in [0, i) of row i
    auto bwd_row = [&](int i, double *r) {
#pragma unroll
        for (int m = 0; m < kInvAhead; ++m) {
            const int k = lane + 64 * m;
            r[m] = (i >= 0 && k < i) ? L[(int64_t)i * n + k] : 0.0;
        }
    };
    bwd_row(n - 1, cur);
    dcur = L[(int64_t)(n - 1) * n + n - 1];
    for (int i = n - 1; i >= 0; --i) {
        bwd_row(i - 1, nxt);
        const double dnxt = i > 0 ? L[(int64_t)(i - 1) * n + i - 1] : 1.0;
        const double xi = y[i] / dcur;
#pragma unroll
        for (int m = 0; m < kInvAhead; ++m) {
            const int k = lane + 64 * m;
            if (k < i) y[k] = y[k] - cur[m] * xi;
        }
        for (int k = lane + 64 * kInvAhead; k < i; k += 64) y[k] = y[k] - L[(int64_t)i * n + k] * xi;
        __syncthreads();
        if (lane == 0) y[i] = xi;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kInvAhead; ++m) cur[m] = nxt[m];
        dcur = dnxt;
    }
    for (int k = lane; k < n; k += 64) X[(int64_t)k * n + j] = y[k];
}


// ------------------------------------------------------------------ FSAI smoother
// Static FSAI factor G (M^{-1} = G^T G, G lower triangular on the pattern of
// the lower triangle of A): row i solves A(P_i, P_i) g = e_last with a dense
// Cholesky factorisation and substitutions, then G(i, P_i) = g / sqrt(g_last).
// The per-entry arithmetic (and its order) is the oracle's: the right-looking
// factorisation and the column-by-column forward substitution apply to each
// entry the same subtractions, in the same order of k, as the oracle's
// row-oriented loops; the backward substitution runs row by row with
// ascending k on one lane, as the oracle's does.

// m_i = number of entries of row i on or below the diagonal; max m into *mmax
__global__ void k_fsai_count(int n, const int32_t *rp, const int32_t *ci, int32_t *cnt, int32_t *mmax) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int m = 0;
    if (i < n) {
        for (int e = rp[i]; e < rp[i + 1]; ++e) m += ci[e] <= i ? 1 : 0;
        cnt[i] = m;
    }
    const unsigned long long bm = block_max_u64<kBlock>((unsigned long long)m);
    if (threadIdx.x == 0) fold_max(mmax, (int32_t)bm);
}

__device__ __forceinline__ double csr_lookup(const int32_t *rp, const int32_t *ci, const double *v, int i, int j) {
    int lo = rp[i], hi = rp[i + 1] - 1;
    while (lo <= hi) {
        const int mid = lo + (hi - lo) / 2;
        if (ci[mid] == j) return v[mid];
        if (ci[mid] < j) lo = mid + 1;
        else hi = mid - 1;
    }
    return 0.0;
}

// TPR threads (one wavefront, or a 256-thread workgroup for long rows) per
// row; the lower triangle of the local matrix packed row by row in LDS:
// entry (r, c), c <= r, at r (r + 1) / 2 + c.
template <int TPR>
__device__ __forceinline__ void fsai_sync() {
    if constexpr (TPR == 64) {
        FSAI_SYNC();
    } else {
        __syncthreads();
    }
}

__device__ __forceinline__ int tri_row(int t) {
    int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    return r;
}

__device__ __forceinline__ int tri_at(int r, int c) { return r * (r + 1) / 2 + c; }

// Right-looking Cholesky of the packed m x m matrix M in place; false (for
// the whole row group) when a pivot is not positive.
template <int TPR>
__device__ bool fsai_factor(double *M, int m, int lane, int *bad) {
    const int tri = m * (m + 1) / 2;
    if (lane == 0) *bad = 0;
    fsai_sync<TPR>();
    for (int k = 0; k < m; ++k) {
        if (lane == 0) {
            const double d = M[tri_at(k, k)];
            if (!(d > 0.0)) *bad = 1;
            else M[tri_at(k, k)] = sqrt(d);
        }
        fsai_sync<TPR>();
        if (*bad) return false;
        const double lkk = M[tri_at(k, k)];
        for (int r = k + 1 + lane; r < m; r += TPR) M[tri_at(r, k)] = M[tri_at(r, k)] / lkk;
        fsai_sync<TPR>();
        for (int t = tri_at(k + 1, 0) + lane; t < tri; t += TPR) {
            const int r = tri_row(t), c = t - r * (r + 1) / 2;
            if (c > k) M[t] = M[t] - M[tri_at(r, k)] * M[tri_at(c, k)];
        }
        fsai_sync<TPR>();
    }
    return true;
}

// y = (L L^T)^{-1} e_last for the factor in M: forward column by column
// (e is overwritten), backward row by row with ascending k on lane 0.
template <int TPR>
__device__ void fsai_solve_last(const double *M, int m, double *e, double *y, int lane) {
    for (int r = lane; r < m; r += TPR) e[r] = r == m - 1 ? 1.0 : 0.0;
    fsai_sync<TPR>();
    for (int k = 0; k < m; ++k) {
        if (lane == 0) e[k] = e[k] / M[tri_at(k, k)];
        fsai_sync<TPR>();
        const double wk = e[k];
        for (int r = k + 1 + lane; r < m; r += TPR) e[r] = e[r] - M[tri_at(r, k)] * wk;
        fsai_sync<TPR>();
    }
    if (lane == 0) {
        for (int r = m - 1; r >= 0; --r) {
            double t = e[r];
            for (int k = r + 1; k < m; ++k) t = t - M[tri_at(k, r)] * y[k];
            y[r] = t / M[tri_at(r, r)];
        }
    }
    fsai_sync<TPR>();
}

template <int MAXM, int WPB, int TPR>
__global__ void __launch_bounds__(WPB * TPR) k_fsai_rows(int n, const int32_t *__restrict__ arp,
                                                         const int32_t *__restrict__ aci,
                                                         const double *__restrict__ av, const int32_t *__restrict__ grp,
                                                         int32_t *gci, double *gv, int32_t *flags) {
    static_assert(TPR == 64 || WPB == 1, "one row per workgroup when a row has more than one wavefront");
    __shared__ double Ms[WPB][MAXM * (MAXM + 1) / 2];
    __shared__ double es[WPB][MAXM], zs[WPB][MAXM];
    __shared__ int idx[WPB][MAXM];
    __shared__ int bad[WPB];
    const int w = threadIdx.x / TPR, lane = threadIdx.x % TPR;
    const int i = blockIdx.x * WPB + w;
    if (i >= n) return;  // the whole row group
    const int m = grp[i + 1] - grp[i];
    if (m < 1 || m > MAXM) {  // uniform over the row group
        if (lane == 0) atomicOr(&flags[6], 1);
        return;
    }
    double *M = Ms[w], *e = es[w], *z = zs[w];
    for (int r = lane; r < m; r += TPR) idx[w][r] = aci[arp[i] + r];
    fsai_sync<TPR>();
    const int tri = m * (m + 1) / 2;
    for (int t = lane; t < tri; t += TPR) {
        const int r = tri_row(t), c = t - r * (r + 1) / 2;
        M[t] = csr_lookup(arp, aci, av, idx[w][r], idx[w][c]);
    }
    fsai_sync<TPR>();
    if (!fsai_factor<TPR>(M, m, lane, &bad[w])) {
        if (lane == 0) atomicOr(&flags[7], 1);
        return;
    }
    fsai_solve_last<TPR>(M, m, e, z, lane);
    if (!(z[m - 1] > 0.0)) {
        if (lane == 0) atomicOr(&flags[7], 1);
        return;
    }
    const double sd = sqrt(z[m - 1]);
    const int o = grp[i];
    for (int r = lane; r < m; r += TPR) {
        gci[o + r] = idx[w][r];
        gv[o + r] = z[r] / sd;
    }
}

// ---------------------------------------------------------------- the paper's interpolations
// Classical (direct coupling a_ij kept in the numerator), extended+i and
// hybrid (Section 2, Interpolation; Alg. extintset).  One row group (a
// wavefront, or a 256-thread workgroup for rows with many candidates)
// builds the interpolatory set of an F row in LDS: candidates are appended,
// then sorted and deduplicated by rank counting.  The weights follow the
// CPU reference's order: the shares of the strong F neighbours are added in
// CSR order of row i, each spread over the set with the sign-filtered
// entries abar_kl of row k (abar_kl = 0 when a_kl has the sign of a_kk), so
// P matches the reference bit for bit.
constexpr int kXiClassical = 1, kXiExt = 2, kXiHybrid = 3;
// candidate capacity of a thread, a wavefront and a 256-thread workgroup (two tiers)
constexpr int kXiCapThread = 32, kXiCapSmall = 128, kXiCapMid = 512, kXiCapGroup = 2048;
// rows handled by one thread: at most kXiCapThread candidates and kXiThreadLen entries
constexpr int kXiThreadLen = 16;

// strong C neighbours of every row
__global__ void k_xi_cs(int n, const int32_t *rp, const int32_t *ci, const uint8_t *strong, const int8_t *cf,
                        int32_t *cs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (ci[e] != i && strong[e] && cf[ci[e]] == kC) ++c;
    cs[i] = c;
}

// upper bound of the candidate list of an F row: |C_i^S|, plus the
// |C_k^S| of its strong F neighbours for the two distance-two variants
__global__ void k_xi_bound(int n, const int32_t *rp, const int32_t *ci, const uint8_t *strong, const int8_t *cf,
                           const int32_t *cs, int variant, int32_t *bnd, unsigned long long *bmax) {
    // bmax[0]: largest bound; bmax[1]: largest bound of the rows that the
    // thread-per-row kernel does not take
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    long long b = 0;
    if (i < n && cf[i] != kC) {
        b = cs[i];
        if (variant != kXiClassical)
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                const int k = ci[e];
                if (k != i && strong[e] && cf[k] == kF) b += cs[k];
            }
    }
    if (i < n) bnd[i] = (int32_t)(b < INT32_MAX ? b : INT32_MAX);
    const bool thread_row = i < n && b <= kXiCapThread && rp[i + 1] - rp[i] <= kXiThreadLen;
    const unsigned long long m = block_max_u64<kBlock>((unsigned long long)b);
    const unsigned long long mw = block_max_u64<kBlock>(thread_row ? 0ull : (unsigned long long)b);
    if (threadIdx.x == 0) {
        fold_max(bmax, m);
        fold_max(bmax + 1, mw);
    }
}

// C rows (identity) and F rows without candidates (empty)
template <bool FILL>
__global__ void k_xi_simple(int n, const int8_t *cf, const int32_t *bnd, const int64_t *cmap, int32_t *cnt,
                            const int32_t *prp, int32_t *pci, double *pv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cf[i] == kC) {
        if constexpr (FILL) {
            pci[prp[i]] = (int32_t)cmap[i];
            pv[prp[i]] = 1.0;
        } else {
            cnt[i] = 1;
        }
    } else if (bnd[i] == 0) {
        if constexpr (!FILL) cnt[i] = 0;
    }
}

template <int CAP, int CAPF, int TPR>
struct XiLds {
    static_assert(16 * CAPF <= 24 * CAP, "the flattened rows overlay the candidate arrays");
    // candidate lists while the set is built; the flattened rows of the
    // fill pass afterwards: column of each entry, its place in the set (-1
    // none, -2 the point i itself) and its sign-filtered value
    union {
        struct {
            int cand[CAP], src[CAP], aux[CAP], pos[CAP], Q[CAP], rem[CAP];
        };
        struct {
            double fab[CAPF];
            int fl[CAPF], fp[CAPF];
        };
    };
    int S[CAP];
    double num[CAP];
    // one chunk (TPR entries) of row i: kind of each entry (0 diagonal, 1
    // strong F neighbour, 2 other member of the set, 3 other), its column and
    // value, and for strong F neighbours the start, length and diagonal of
    // their row
    int mk[TPR], mkind[TPR], mr0[TPR], mlen[TPR];
    double ma[TPR], makk[TPR];
    // a group of consecutive chunk entries whose strong F rows, laid end to
    // end, fit CAPF entries: chunk position and offset of each such row
    int gq[TPR], goff[TPR + 1], gb[TPR], hasc[TPR], cov[TPR];
    double gD[TPR], gai[TPR];  // denominators of the group's rows, their sign-filtered entry at i
    double red[TPR / 64];
    int redi[TPR / 64];
    unsigned long long redu[TPR / 64];
    double term[TPR];
    double diag;
    int cnt;
};

template <int TPR>
__device__ __forceinline__ double xi_sum(double x, double *red, int lane) {
    x = wave_sum(x);
    if constexpr (TPR == 64) {
        return x;
    } else {
        __syncthreads();
        if ((lane & 63) == 0) red[lane >> 6] = x;
        __syncthreads();
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < TPR / 64; ++w) t += red[w];
        __syncthreads();
        return t;
    }
}

template <int TPR>
__device__ __forceinline__ int xi_sum_i(int x, int *red, int lane) {
    x = wave_sum_i(x);
    if constexpr (TPR == 64) {
        return x;
    } else {
        __syncthreads();
        if ((lane & 63) == 0) red[lane >> 6] = x;
        __syncthreads();
        int t = 0;
#pragma unroll
        for (int w = 0; w < TPR / 64; ++w) t += red[w];
        __syncthreads();
        return t;
    }
}

template <int TPR>
__device__ __forceinline__ unsigned long long xi_max(unsigned long long x, unsigned long long *red, int lane) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, kWave);
        x = y > x ? y : x;
    }
    if constexpr (TPR == 64) {
        return x;
    } else {
        __syncthreads();
        if ((lane & 63) == 0) red[lane >> 6] = x;
        __syncthreads();
        unsigned long long t = 0;
#pragma unroll
        for (int w = 0; w < TPR / 64; ++w) t = red[w] > t ? red[w] : t;
        __syncthreads();
        return t;
    }
}

// position of c in the ascending S[0, U) or -1
__device__ __forceinline__ int xi_find(const int *S, int U, int c) {
    int lo = 0, hi = U - 1;
    while (lo <= hi) {
        const int mid = lo + ((hi - lo) >> 1);
        const int x = S[mid];
        if (x == c) return mid;
        if (x < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// Exclusive scan of one int per lane over the row group; *total gets the sum.
template <int TPR>
__device__ __forceinline__ int xi_scan_excl(int c, int *red, int lane, int *total) {
    int x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, kWave);
        if ((lane & 63) >= o) x += y;
    }
    if constexpr (TPR == 64) {
        *total = __shfl(x, 63, kWave);
        return x - c;
    } else {
        __syncthreads();
        if ((lane & 63) == 63) red[lane >> 6] = x;
        __syncthreads();
        int base = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < TPR / 64; ++w) {
            if (w < (lane >> 6)) base += red[w];
            tot += red[w];
        }
        __syncthreads();
        *total = tot;
        return base + x - c;
    }
}

// ------------------------------------------------------------------ adaptive FSAI
// Row i of the adaptive factor minimises psi_i(g) = g^T A g (g_i = 1) over a
// pattern P_i grown from {i} (Section 2, eq. smo; the pattern search of the
// FSAI package the paper cites).  Each pass solves A(P, P) y = e_last
// (psi = 1 / y_last); the row stops after `steps` growth steps or when psi
// fell by no more than eps times its previous value; otherwise the `step`
// candidates j < i (columns of the rows indexed by P, outside P) with the
// largest |z_j|, z_j = sum over row j of a_jc y_c for c in P (the Kaporin
// gradient up to a positive factor), join P, the smaller j first on ties.
// G(i, P_i) = y / sqrt(y_last).  Every rounding is the oracle's: the local
// solves as in k_fsai_rows, z_j summed along row j in CSR order.
//
// One wavefront per row.  The candidate set is kept sorted in LDS and
// updated between passes (members that joined P leave it, the rows of the
// new members are merged in), at most CAP entries: the largest tier
// (kAfsaiMaxCand) raises flags[6] on overflow, and the level falls back to
// Jacobi; a smaller tier is launched only where the bound
// (steps * step + 1) * max row length rules overflow out (flags[4]
// otherwise).  Rows are written padded (mcap slots each) with their counts.
constexpr int kAfsaiMaxM = 32, kAfsaiMaxCand = 2048;

// number of entries of the ascending S[0, len) below x
__device__ __forceinline__ int afsai_below(const int *S, int len, int x) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (S[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int wave_min_i(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(x, o, kWave);
        x = y < x ? y : x;
    }
    return x;
}

template <int MAXM, int CAP, int WPB>
__global__ void __launch_bounds__(WPB * 64) k_afsai_rows(int n, const int32_t *__restrict__ arp,
                                                         const int32_t *__restrict__ aci,
                                                         const double *__restrict__ av,
                                                         const int32_t *__restrict__ tpos, int steps, int step,
                                                         double eps, int mcap, int32_t *__restrict__ cnt,
                                                         int32_t *__restrict__ pci, double *__restrict__ pv,
                                                         int32_t *flags) {
    constexpr int Q = CAP / 64;
    __shared__ double Ms[WPB][MAXM * (MAXM + 1) / 2];
    __shared__ double es[WPB][MAXM], ys[WPB][MAXM];
    __shared__ int Ps[WPB][MAXM], pends[WPB][MAXM];
    // candidates (C), then two work lists (T, N) that the scattered gradient
    // of the large tiers reuses as CAP doubles once the candidates are merged
    __shared__ __align__(16) int cbuf[WPB][3][CAP];
    __shared__ int bad[WPB];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * WPB + w;
    if (i >= n) return;  // the whole wavefront
    double *M = Ms[w], *e = es[w], *y = ys[w];
    int *P = Ps[w], *pend = pends[w];
    int *C = cbuf[w][0], *T = cbuf[w][1], *N = cbuf[w][2];
    int m = 1, nC = 0, npend = 1;
    if (lane == 0) {
        P[0] = i;
        pend[0] = i;
    }
    FSAI_SYNC();
    double psi_prev = 0.0;
    double zr[CAP <= 256 ? Q : 1];  // the small tier's gradient, one candidate per lane and slot
    for (int k = 0;; ++k) {
        // 1. local system A(P, P) y = e_last; row r of the local matrix from
        //    row P[r] of A, matched against P[0..r]
        const int tri = m * (m + 1) / 2;
        for (int t = lane; t < tri; t += 64) M[t] = 0.0;
        FSAI_SYNC();
        if (lane < m) {
            const int r = lane, row = P[r];
            int c = 0;
            for (int q = arp[row]; q < arp[row + 1] && c <= r; ++q) {
                const int col = aci[q];
                while (c <= r && P[c] < col) ++c;
                if (c <= r && P[c] == col) M[tri_at(r, c)] = av[q];
            }
        }
        FSAI_SYNC();
        if (!fsai_factor<64>(M, m, lane, &bad[w])) {
            if (lane == 0) atomicOr(&flags[7], 1);
            return;
        }
        fsai_solve_last<64>(M, m, e, y, lane);
        const double ylast = y[m - 1];
        if (!(ylast > 0.0)) {
            if (lane == 0) atomicOr(&flags[7], 1);
            return;
        }
        // 2. stopping tests
        const double psi = 1.0 / ylast;
        if (k == steps) break;
        if (k > 0 && psi_prev - psi <= eps * psi_prev) break;
        psi_prev = psi;
        // 3. candidate set: the new members leave it, their rows join it
        if (k > 0) {
            int nk = 0;
            for (int b = 0; b < nC; b += 64) {
                const int idx = b + lane;
                const int c = idx < nC ? C[idx] : -1;
                bool keep = idx < nC;
                for (int a = 0; a < npend; ++a) keep = keep && pend[a] != c;
                int tot;
                const int off = xi_scan_excl<64>(keep ? 1 : 0, nullptr, lane, &tot);
                if (keep) T[nk + off] = c;
                nk += tot;
            }
            FSAI_SYNC();
            for (int t = lane; t < nk; t += 64) C[t] = T[t];
            FSAI_SYNC();
            nC = nk;
        }
        for (int a = 0; a < npend; ++a) {
            const int q = pend[a], rs = arp[q], re = arp[q + 1];
            int nN = 0;
            for (int b = rs; b < re; b += 64) {
                if (aci[b] >= i) break;  // rows are sorted: nothing below i is left
                const int ee = b + lane;
                const int j = ee < re ? aci[ee] : INT_MAX;
                const bool keep = j < i && xi_find(P, m, j) < 0 && xi_find(C, nC, j) < 0;
                int tot;
                const int off = xi_scan_excl<64>(keep ? 1 : 0, nullptr, lane, &tot);
                if (nC + nN + tot > CAP) {
                    if (lane == 0) atomicOr(&flags[CAP == kAfsaiMaxCand ? 6 : 4], 1);
                    return;
                }
                if (keep) N[nN + off] = j;
                nN += tot;
            }
            FSAI_SYNC();
            if (nN > 0) {
                for (int idx = lane; idx < nC; idx += 64) {
                    const int c = C[idx];
                    T[idx + afsai_below(N, nN, c)] = c;
                }
                for (int idx = lane; idx < nN; idx += 64) {
                    const int x = N[idx];
                    T[idx + afsai_below(C, nC, x)] = x;
                }
                FSAI_SYNC();
                for (int t = lane; t < nC + nN; t += 64) C[t] = T[t];
                FSAI_SYNC();
                nC += nN;
            }
        }
        npend = 0;
        // gradient components z_j = sum over c in P of a_jc y_c, each added
        // in ascending c from 0.0 (the sum along row j of A in CSR order).
        // Small candidate sets (short rows): each lane walks the rows of its
        // candidates.  Large ones: the terms are scattered from the rows of
        // the pattern instead (|P| rows rather than every candidate's): for
        // c = P[0], P[1], ... in turn the lanes take the entries (c, j) of
        // row c with j < i, and a candidate j adds a_jc (its own row's value,
        // at the transpose position) times y_c -- the same terms in the same
        // order, so both ways round alike.
        if constexpr (CAP <= 256) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int idx = lane + 64 * q;
                double sz = 0.0;
                if (idx < nC) {
                    const int j = C[idx];
                    int pp = 0;
                    for (int t = arp[j]; t < arp[j + 1]; ++t) {
                        const int col = aci[t];
                        if (col > i) break;
                        while (pp < m && P[pp] < col) ++pp;
                        if (pp < m && P[pp] == col) sz = sz + av[t] * y[pp];
                    }
                }
                zr[q] = sz;
            }
        } else {
            double *z = reinterpret_cast<double *>(cbuf[w][1]);  // over T and N
            for (int t = lane; t < nC; t += 64) z[t] = 0.0;
            FSAI_SYNC();
            for (int r = 0; r < m; ++r) {
                const int c = P[r], ce = arp[c + 1];
                const double yc = y[r];
                for (int b = arp[c]; b < ce; b += 64) {
                    if (aci[b] >= i) break;  // rows are sorted: nothing below i is left
                    const int e = b + lane;
                    const int j = e < ce ? aci[e] : INT_MAX;
                    if (j < i) {
                        const int slot = xi_find(C, nC, j);
                        if (slot >= 0) z[slot] = z[slot] + av[tpos[e]] * yc;
                    }
                }
                FSAI_SYNC();
            }
        }
        // 4. the `step` largest |z_j| > 0 join P (smaller j on ties: C is ascending)
        double *zl = reinterpret_cast<double *>(cbuf[w][1]);  // the large tiers' gradient
        for (int a = 0; a < step; ++a) {
            unsigned long long best = 0;
            int bidx = INT_MAX;
            if constexpr (CAP <= 256) {
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(zr[q]));
                    if (bits > best) {
                        best = bits;
                        bidx = lane + 64 * q;
                    }
                }
            } else {
                for (int idx = lane; idx < nC; idx += 64) {
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(zl[idx]));
                    if (bits > best) {
                        best = bits;
                        bidx = idx;
                    }
                }
            }
            const unsigned long long top = xi_max<64>(best, nullptr, lane);
            if (top == 0) break;
            const int widx = wave_min_i(best == top ? bidx : INT_MAX);
            if constexpr (CAP <= 256) {
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    if (lane + 64 * q == widx) zr[q] = 0.0;
            } else if (lane == 0) {
                zl[widx] = 0.0;
            }
            if (lane == 0) {
                const int j = C[widx];
                int r = m;
                while (r > 0 && P[r - 1] > j) {
                    P[r] = P[r - 1];
                    --r;
                }
                P[r] = j;
                pend[npend] = j;
            }
            ++m;
            ++npend;
            FSAI_SYNC();
        }
        if (npend == 0) break;
    }
    const double sd = sqrt(y[m - 1]);
    for (int r = lane; r < m; r += 64) {
        pci[(int64_t)i * mcap + r] = P[r];
        pv[(int64_t)i * mcap + r] = y[r] / sd;
    }
    if (lane == 0) cnt[i] = m;
}

// padded rows -> CSR (G.rp already the scan of the counts)
__global__ void k_afsai_compact(int n, int mcap, const int32_t *pci, const double *pv, const int32_t *grp,
                                int32_t *gci, double *gv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int o = grp[i], m = grp[i + 1] - o;
    for (int r = 0; r < m; ++r) {
        gci[o + r] = pci[(int64_t)i * mcap + r];
        gv[o + r] = pv[(int64_t)i * mcap + r];
    }
}

// The distinct values of key[0, T) in ascending order go to out[0, U);
// pos[t] is the place of key[t] in out (when pos is given); returns U (all
// lanes).  Short lists are ranked in place (key keeps its order; `first` is
// scratch); longer ones are bitonic-sorted in place first (key, and tag
// with it when given, then hold the sorted order) and deduplicated with a
// scan.  key must have room for the next power of two of T entries.
template <int TPR>
__device__ int xi_sort_unique(int *key, int *tag, int T, int *out, int *pos, int *first, int *red, int lane) {
    if (T <= 64) {
        for (int t = lane; t < T; t += TPR) {
            const int x = key[t];
            int f = 1;
            for (int u = 0; u < t; ++u)
                if (key[u] == x) {
                    f = 0;
                    break;
                }
            first[t] = f;
        }
        fsai_sync<TPR>();
        int mine = 0;
        for (int t = lane; t < T; t += TPR) {
            const int x = key[t];
            int r = 0;
            for (int u = 0; u < T; ++u) r += (first[u] && key[u] < x) ? 1 : 0;
            if (pos) pos[t] = r;
            if (first[t]) {
                out[r] = x;
                ++mine;
            }
        }
        fsai_sync<TPR>();
        return xi_sum_i<TPR>(mine, red, lane);
    }
    int np = 64;
    while (np < T) np <<= 1;
    for (int t = T + lane; t < np; t += TPR) key[t] = INT_MAX;
    fsai_sync<TPR>();
    for (int kk = 2; kk <= np; kk <<= 1) {
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int t = lane; t < np; t += TPR) {
                const int u = t ^ jj;
                if (u > t) {
                    const int x = key[t], y = key[u];
                    const bool up = (t & kk) == 0;
                    if (up ? (x > y) : (x < y)) {
                        key[t] = y;
                        key[u] = x;
                        if (tag) {
                            const int g = tag[t];
                            tag[t] = tag[u];
                            tag[u] = g;
                        }
                    }
                }
            }
            fsai_sync<TPR>();
        }
    }
    // contiguous segments per lane: count the first entries of each value,
    // scan, then place them
    const int seg = (T + TPR - 1) / TPR, t0 = min(T, lane * seg), t1 = min(T, t0 + seg);
    int c = 0;
    for (int t = t0; t < t1; ++t) c += (t == 0 || key[t] != key[t - 1]) ? 1 : 0;
    int U;
    int run = xi_scan_excl<TPR>(c, red, lane, &U);
    for (int t = t0; t < t1; ++t) {
        if (t == 0 || key[t] != key[t - 1]) out[run++] = key[t];
        if (pos) pos[t] = run - 1;
    }
    fsai_sync<TPR>();
    return U;
}

// strong C neighbours of row k appended to cand (with source b when hybrid)
template <int CAP, int CAPF, int TPR>
__device__ __forceinline__ void xi_append(XiLds<CAP, CAPF, TPR> &G, const int32_t *rp, const int32_t *ci,
                                          const uint8_t *strong, const int8_t *cf, int k, int b, int lane) {
    for (int f = rp[k] + lane; f < rp[k + 1]; f += TPR) {
        const int c = ci[f];
        if (c != k && strong[f] && cf[c] == kC) {
            const int t = atomicAdd(&G.cnt, 1);
            if (t < CAP) {
                G.cand[t] = c;
                G.src[t] = b;
            }
        }
    }
}

// metadata of entries [eb, eb + me) of row i (set membership tested when
// U >= 0; values and the neighbours' diagonals loaded when vals)
template <int CAP, int CAPF, int TPR>
__device__ __forceinline__ void xi_meta(XiLds<CAP, CAPF, TPR> &G, int i, int eb, int me, const int32_t *rp,
                                        const int32_t *ci, const double *v, const uint8_t *strong, const int8_t *cf,
                                        int U, bool vals, int lane) {
    if (lane < me) {
        const int e = eb + lane, k = ci[e];
        int kind = 3, r0 = 0, len = 0;
        double akk = 0.0;
        if (k == i) {
            kind = 0;
        } else if (strong[e] && cf[k] == kF) {
            kind = 1;
            r0 = rp[k];
            len = rp[k + 1] - r0;
            if (vals) akk = csr_lookup(rp, ci, v, k, k);
        } else if (U >= 0 && xi_find(G.S, U, k) >= 0) {
            kind = 2;
        }
        G.mk[lane] = k;
        G.mkind[lane] = kind;
        G.mr0[lane] = r0;
        G.mlen[lane] = len;
        G.makk[lane] = akk;
        G.ma[lane] = vals ? v[e] : 0.0;
    }
    fsai_sync<TPR>();
}

// The group of chunk entries [q, qb) whose strong F rows fit CAPF entries
// end to end: gq/goff list those rows (nk of them, tot entries).  nk == 0
// with qb < me means entry qb alone is a longer row.
template <int CAP, int CAPF, int TPR>
__device__ __forceinline__ int xi_group(XiLds<CAP, CAPF, TPR> &G, int q, int me, int lane, int &nk, int &tot) {
    int qb = q;
    nk = 0;
    tot = 0;
    while (qb < me) {
        if (G.mkind[qb] == 1) {
            const int ln = G.mlen[qb];
            if (tot + ln > CAPF) break;
            if (lane == 0) {
                G.gq[nk] = qb;
                G.goff[nk] = tot;
            }
            ++nk;
            tot += ln;
        }
        ++qb;
    }
    if (lane == 0) G.goff[nk] = tot;
    fsai_sync<TPR>();
    return qb;
}

// row of the group holding flattened entry t (the largest j with goff[j] <= t)
__device__ __forceinline__ int xi_seg(const int *goff, int nk, int t) {
    int lo = 0, hi = nk - 1;
    while (lo < hi) {
        const int mid = lo + ((hi - lo + 1) >> 1);
        if (goff[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double xi_abar(double x, int sd) {
    const int sx = (x > 0.0) - (x < 0.0);
    return sx == sd ? 0.0 : x;
}

// share of one strong F neighbour k whose row is longer than CAPF: its
// entries are read from global memory in chunks (same operations and order
// as the grouped path); returns the new diagonal
template <int CAP, int CAPF, int TPR>
__device__ double xi_share_long(XiLds<CAP, CAPF, TPR> &G, int i, int k, double a, double akk, bool plus_i, int U,
                                double diag, const int32_t *rp, const int32_t *ci, const double *v, int lane) {
    const int f0 = rp[k], f1 = rp[k + 1];
    const int sd = (akk > 0.0) - (akk < 0.0);
    double D = 0.0;
    for (int fb = f0; fb < f1; fb += TPR) {
        const int f = fb + lane;
        double term = 0.0;
        if (f < f1) {
            const int l = ci[f];
            if ((plus_i && l == i) || xi_find(G.S, U, l) >= 0) term = xi_abar(v[f], sd);
        }
        G.term[lane] = term;
        fsai_sync<TPR>();
        const int m = min(TPR, f1 - fb);
        for (int q = 0; q < m; ++q) D = D + G.term[q];
        fsai_sync<TPR>();
    }
    if (D == 0.0) return diag + a;
    double dt = 0.0;
    for (int f = f0 + lane; f < f1; f += TPR) {
        const int l = ci[f];
        const double ab = xi_abar(v[f], sd);
        if (l == i) {
            if (plus_i) dt = (a * ab) / D;
        } else {
            const int p = xi_find(G.S, U, l);
            if (p >= 0) G.num[p] = G.num[p] + (a * ab) / D;
        }
    }
    dt = xi_sum<TPR>(dt, G.red, lane);
    fsai_sync<TPR>();
    return plus_i ? diag + dt : diag;
}

// Rows with at most MAXT candidates: one thread per row runs the CPU
// reference's loops directly, with the set and the numerators in private
// arrays (same operations, same order, so the same bits).
__device__ __forceinline__ bool xi_depends(const int32_t *rp, const int32_t *ci, const uint8_t *strong, int k, int l) {
    const int e = find_col(ci, rp[k], rp[k + 1], l);
    return e >= 0 && strong[e];
}

template <int MAXT, bool FILL>
__global__ void __launch_bounds__(256)
    k_xi_thread(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ v,
                const uint8_t *__restrict__ strong, const int8_t *__restrict__ cf, const int32_t *__restrict__ bnd,
                int variant, const int64_t *__restrict__ cmap, int32_t *cnt, const int32_t *__restrict__ prp,
                int32_t *pci, double *pv, int32_t *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || cf[i] == kC) return;
    const int bi = bnd[i];
    if (bi < 1 || bi > MAXT) return;
    const int e0 = rp[i], e1 = rp[i + 1];
    if (e1 - e0 > kXiThreadLen) return;
    int set[MAXT];
    int m = 0;
    auto in_set = [&](int c) {
        for (int t = 0; t < m; ++t)
            if (set[t] == c) return true;
        return false;
    };
    for (int e = e0; e < e1; ++e) {
        const int c = ci[e];
        if (c != i && strong[e] && cf[c] == kC) set[m++] = c;  // ascending
    }
    const int s0 = m;
    if (variant == kXiExt) {
        for (int e = e0; e < e1; ++e) {
            const int k = ci[e];
            if (k == i || !strong[e] || cf[k] != kF) continue;
            for (int f = rp[k]; f < rp[k + 1]; ++f) {
                const int c = ci[f];
                if (c != k && strong[f] && cf[c] == kC && !in_set(c)) set[m++] = c;
            }
        }
    } else if (variant == kXiHybrid) {
        int fp[MAXT];
        int nf = 0;
        for (int e = e0; e < e1; ++e) {
            const int k = ci[e];
            if (k == i || !strong[e] || cf[k] != kF) continue;
            bool has_c = false, covered = false;
            for (int f = rp[k]; f < rp[k + 1]; ++f) {
                const int c = ci[f];
                if (c == k || !strong[f] || cf[c] != kC) continue;
                has_c = true;
                for (int t = 0; t < s0; ++t)
                    if (set[t] == c) covered = true;
            }
            if (has_c && !covered) fp[nf++] = k;  // nf <= bound <= MAXT
        }
        while (nf > 0) {
            int best = -1, bestdeg = 0;
            for (int a = 0; a < nf; ++a) {
                const int k = fp[a];
                for (int f = rp[k]; f < rp[k + 1]; ++f) {
                    const int c = ci[f];
                    if (c == k || !strong[f] || cf[c] != kC) continue;
                    int deg = 0;
                    for (int b = 0; b < nf; ++b) deg += xi_depends(rp, ci, strong, fp[b], c) ? 1 : 0;
                    if (deg > bestdeg || (deg == bestdeg && c < best)) {
                        best = c;
                        bestdeg = deg;
                    }
                }
            }
            set[m++] = best;
            int keep = 0;
            for (int a = 0; a < nf; ++a)
                if (!xi_depends(rp, ci, strong, fp[a], best)) fp[keep++] = fp[a];
            nf = keep;
        }
    }
    // ascending order (insertion sort)
    for (int t = 1; t < m; ++t) {
        const int x = set[t];
        int u = t - 1;
        while (u >= 0 && set[u] > x) {
            set[u + 1] = set[u];
            --u;
        }
        set[u + 1] = x;
    }
    if constexpr (!FILL) {
        cnt[i] = m;
        return;
    } else {
        const int o = prp[i];
        if (prp[i + 1] - o != m) {
            atomicOr(&flags[1], 1);
            return;
        }
        auto pos_of = [&](int c) {
            int lo = 0, hi = m - 1;
            while (lo <= hi) {
                const int mid = lo + ((hi - lo) >> 1);
                if (set[mid] == c) return mid;
                if (set[mid] < c) lo = mid + 1;
                else hi = mid - 1;
            }
            return -1;
        };
        const bool plus_i = variant != kXiClassical;
        double num[MAXT];
        for (int t = 0; t < m; ++t) num[t] = 0.0;
        double diag = 0.0;
        for (int e = e0; e < e1; ++e) {
            const int c = ci[e];
            if (c == i) diag = v[e];
            else {
                const int p = pos_of(c);
                if (p >= 0) num[p] = v[e];
            }
        }
        for (int e = e0; e < e1; ++e) {
            const int k = ci[e];
            if (k == i) continue;
            const double a = v[e];
            if (strong[e] && cf[k] == kF) {
                const int f0 = rp[k], f1 = rp[k + 1];
                const double akk = csr_lookup(rp, ci, v, k, k);
                const int sd = (akk > 0.0) - (akk < 0.0);
                double D = 0.0;
                for (int f = f0; f < f1; ++f) {
                    const int l = ci[f];
                    if ((plus_i && l == i) || pos_of(l) >= 0) D = D + xi_abar(v[f], sd);
                }
                if (D == 0.0) {
                    diag = diag + a;
                    continue;
                }
                for (int f = f0; f < f1; ++f) {
                    const int l = ci[f];
                    const double ab = xi_abar(v[f], sd);
                    if (l == i) {
                        if (plus_i) diag = diag + (a * ab) / D;
                    } else {
                        const int p = pos_of(l);
                        if (p >= 0) num[p] = num[p] + (a * ab) / D;
                    }
                }
            } else if (pos_of(k) < 0) {
                diag = diag + a;  // weak neighbour outside the set
            }
        }
        for (int t = 0; t < m; ++t) {
            pci[o + t] = (int32_t)cmap[set[t]];
            pv[o + t] = -num[t] / diag;
        }
    }
}

// flags[0]: candidate list longer than the row group's capacity;
// flags[1]: the fill pass found another set size than the count pass
template <int CAP, int CAPF, int WPB, int TPR, bool FILL>
__global__ void __launch_bounds__(WPB * TPR)
    k_xi_rows(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ v,
              const uint8_t *__restrict__ strong, const int8_t *__restrict__ cf, const int32_t *__restrict__ bnd,
              int lo, int hi, int variant, const int64_t *__restrict__ cmap, int32_t *cnt,
              const int32_t *__restrict__ prp, int32_t *pci, double *pv, int32_t *flags) {
    static_assert(TPR == 64 || WPB == 1, "one row per workgroup when a row has more than one wavefront");
    __shared__ XiLds<CAP, CAPF, TPR> Ls[WPB];
    const int w = threadIdx.x / TPR, lane = threadIdx.x % TPR;
    const int i = blockIdx.x * WPB + w;
    if (i >= n || cf[i] == kC) return;  // uniform over the row group
    const int bi = bnd[i];
    if (bi < lo || bi > hi) return;
    const int e0 = rp[i], e1 = rp[i + 1];
    if (bi <= kXiCapThread && e1 - e0 <= kXiThreadLen) return;  // one thread per row (k_xi_thread)
    XiLds<CAP, CAPF, TPR> &G = Ls[w];
    // C_i^S, and for extended+i the strong C neighbours of the strong F
    // neighbours (their rows loaded end to end, a group at a time)
    if (lane == 0) G.cnt = 0;
    fsai_sync<TPR>();
    xi_append<CAP, CAPF, TPR>(G, rp, ci, strong, cf, i, 0, lane);
    if (variant == kXiExt) {
        for (int eb = e0; eb < e1; eb += TPR) {
            const int me = min(TPR, e1 - eb);
            xi_meta<CAP, CAPF, TPR>(G, i, eb, me, rp, ci, v, strong, cf, -1, false, lane);
            for (int q = 0; q < me;) {
                int nk, tot;
                const int qb = xi_group<CAP, CAPF, TPR>(G, q, me, lane, nk, tot);
                if (nk == 0) {
                    if (qb < me) xi_append<CAP, CAPF, TPR>(G, rp, ci, strong, cf, G.mk[qb], 0, lane);
                    q = qb + 1;
                    fsai_sync<TPR>();
                    continue;
                }
                for (int t = lane; t < tot; t += TPR) {
                    const int j = xi_seg(G.goff, nk, t), qq = G.gq[j];
                    const int f = G.mr0[qq] + (t - G.goff[j]), k = G.mk[qq];
                    const int c = ci[f];
                    if (c != k && strong[f] && cf[c] == kC) {
                        const int s2 = atomicAdd(&G.cnt, 1);
                        if (s2 < CAP) G.cand[s2] = c;
                    }
                }
                fsai_sync<TPR>();
                q = qb;
            }
        }
    }
    fsai_sync<TPR>();
    const int T = G.cnt;
    if (T > CAP) {
        if (lane == 0) atomicOr(&flags[0], 1);
        return;
    }
    int U = xi_sort_unique<TPR>(G.cand, nullptr, T, G.S, nullptr, G.aux, G.redi, lane);
    if (variant == kXiHybrid) {
        // Alg. extintset: F' = strong F neighbours with a strong C neighbour
        // but none in C_i^S (numbered in CSR order); candidates = their
        // strong C neighbours, tagged with the F' point they cover
        const int s0 = U;
        int nf = 0;
        if (lane == 0) G.cnt = 0;
        fsai_sync<TPR>();
        for (int eb = e0; eb < e1; eb += TPR) {
            const int me = min(TPR, e1 - eb);
            xi_meta<CAP, CAPF, TPR>(G, i, eb, me, rp, ci, v, strong, cf, -1, false, lane);
            for (int q = 0; q < me;) {
                int nk, tot;
                const int qb = xi_group<CAP, CAPF, TPR>(G, q, me, lane, nk, tot);
                if (nk == 0) {
                    if (qb < me) {  // one long row
                        const int k = G.mk[qb];
                        int hasc = 0, cov = 0;
                        for (int f = rp[k] + lane; f < rp[k + 1]; f += TPR) {
                            const int c = ci[f];
                            if (c != k && strong[f] && cf[c] == kC) {
                                hasc = 1;
                                if (xi_find(G.S, s0, c) >= 0) cov = 1;
                            }
                        }
                        hasc = xi_sum_i<TPR>(hasc, G.redi, lane);
                        cov = xi_sum_i<TPR>(cov, G.redi, lane);
                        if (hasc != 0 && cov == 0) {
                            xi_append<CAP, CAPF, TPR>(G, rp, ci, strong, cf, k, nf, lane);
                            if (lane == 0 && nf < CAP) G.rem[nf] = 1;
                            ++nf;
                        }
                    }
                    q = qb + 1;
                    fsai_sync<TPR>();
                    continue;
                }
                for (int j = lane; j < nk; j += TPR) {
                    G.hasc[j] = 0;
                    G.cov[j] = 0;
                }
                fsai_sync<TPR>();
                for (int t = lane; t < tot; t += TPR) {
                    const int j = xi_seg(G.goff, nk, t), qq = G.gq[j];
                    const int f = G.mr0[qq] + (t - G.goff[j]), k = G.mk[qq];
                    const int c = ci[f];
                    if (c != k && strong[f] && cf[c] == kC) {
                        G.hasc[j] = 1;
                        if (xi_find(G.S, s0, c) >= 0) G.cov[j] = 1;
                    }
                }
                fsai_sync<TPR>();
                for (int j = 0; j < nk; ++j) {  // uniform: every lane numbers F' alike
                    int b = -1;
                    if (G.hasc[j] && !G.cov[j]) {
                        b = nf;
                        if (lane == 0 && nf < CAP) G.rem[nf] = 1;
                        ++nf;
                    }
                    if (lane == 0) G.gb[j] = b;
                }
                fsai_sync<TPR>();
                for (int t = lane; t < tot; t += TPR) {
                    const int j = xi_seg(G.goff, nk, t);
                    const int b = G.gb[j];
                    if (b < 0) continue;
                    const int qq = G.gq[j];
                    const int f = G.mr0[qq] + (t - G.goff[j]), k = G.mk[qq];
                    const int c = ci[f];
                    if (c != k && strong[f] && cf[c] == kC) {
                        const int s2 = atomicAdd(&G.cnt, 1);
                        if (s2 < CAP) {
                            G.cand[s2] = c;
                            G.src[s2] = b;
                        }
                    }
                }
                fsai_sync<TPR>();
                q = qb;
            }
        }
        fsai_sync<TPR>();
        const int T2 = G.cnt;
        if (T2 > CAP || s0 + nf > CAP) {
            if (lane == 0) atomicOr(&flags[0], 1);
            return;
        }
        if (nf > 0) {
            const int U2 = xi_sort_unique<TPR>(G.cand, G.src, T2, G.Q, G.pos, G.aux, G.redi, lane);
            int np = 0;
            for (;;) {
                // degree of each candidate over the points of F' still uncovered
                for (int u = lane; u < U2; u += TPR) G.aux[u] = 0;
                fsai_sync<TPR>();
                for (int t = lane; t < T2; t += TPR)
                    if (G.rem[G.src[t]]) atomicAdd(&G.aux[G.pos[t]], 1);
                fsai_sync<TPR>();
                unsigned long long key = 0;
                for (int u = lane; u < U2; u += TPR) {
                    const int d = G.aux[u];
                    const unsigned long long kk =
                        d > 0 ? ((unsigned long long)d << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)G.Q[u])
                              : 0ull;
                    key = kk > key ? kk : key;
                }
                key = xi_max<TPR>(key, G.redu, lane);
                if (key == 0) break;
                // most points covered, smallest index on ties
                const int cstar = (int)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
                if (lane == 0) G.S[s0 + np] = cstar;
                ++np;
                for (int t = lane; t < T2; t += TPR)
                    if (G.cand[t] == cstar) G.rem[G.src[t]] = 0;
                fsai_sync<TPR>();
            }
            U = s0 + np;
            fsai_sync<TPR>();
            for (int u = lane; u < U; u += TPR) G.cand[u] = G.S[u];
            fsai_sync<TPR>();
            xi_sort_unique<TPR>(G.cand, nullptr, U, G.S, nullptr, G.aux, G.redi, lane);
        }
    }
    if constexpr (!FILL) {
        if (lane == 0) cnt[i] = U;
        return;
    } else {
        const int o = prp[i];
        if (prp[i + 1] - o != U) {
            if (lane == 0) atomicOr(&flags[1], 1);
            return;
        }
        const bool plus_i = variant != kXiClassical;
        for (int u = lane; u < U; u += TPR) G.num[u] = 0.0;
        fsai_sync<TPR>();
        for (int e = e0 + lane; e < e1; e += TPR) {
            const int c = ci[e];
            if (c == i) {
                G.diag = v[e];
            } else {
                const int p = xi_find(G.S, U, c);
                if (p >= 0) G.num[p] = v[e];
            }
        }
        fsai_sync<TPR>();
        double diag = G.diag;
        // row i in CSR order: weak neighbours outside the set go to the
        // diagonal; each strong F neighbour k spreads a_ik over the set (and
        // i itself unless classical) in proportion to the sign-filtered
        // entries of its row, whose denominator is added in ascending column
        // order -- the CPU reference's operations in its order.  The rows of
        // a group of neighbours are loaded together; the sums run in LDS.
        for (int eb = e0; eb < e1; eb += TPR) {
            const int me = min(TPR, e1 - eb);
            xi_meta<CAP, CAPF, TPR>(G, i, eb, me, rp, ci, v, strong, cf, U, true, lane);
            for (int q = 0; q < me;) {
                int nk, tot;
                const int qb = xi_group<CAP, CAPF, TPR>(G, q, me, lane, nk, tot);
                // four entries per lane at a time: their row lookups, loads
                // and set searches run in lockstep so the latencies overlap
                {
                    int sstep = 1, gstep = 1;
                    while (sstep * 2 <= U) sstep *= 2;
                    while (gstep * 2 <= nk) gstep *= 2;
                    for (int t0 = lane; t0 < tot; t0 += 4 * TPR) {
                        int tt[4], f[4], l[4], jr[4], lo[4];
                        double x[4], akk[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            tt[r] = t0 + r * TPR;
                            jr[r] = 0;
                        }
                        // row of the group: the largest j with goff[j] <= t
                        for (int st = gstep; st > 0; st >>= 1) {
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                if (jr[r] + st < nk && G.goff[jr[r] + st] <= tt[r]) jr[r] += st;
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const bool ok = tt[r] < tot;
                            const int qq = G.gq[jr[r]];
                            f[r] = ok ? G.mr0[qq] + (tt[r] - G.goff[jr[r]]) : G.mr0[qq];
                            akk[r] = G.makk[qq];
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            l[r] = ci[f[r]];
                            x[r] = v[f[r]];
                            lo[r] = 0;
                        }
                        // lower bound of l in the set
                        for (int st = sstep; st > 0; st >>= 1) {
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                if (lo[r] + st <= U && G.S[lo[r] + st - 1] < l[r]) lo[r] += st;
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            if (tt[r] >= tot) continue;
                            const int pp = (lo[r] < U && G.S[lo[r]] == l[r]) ? lo[r] : -1;
                            G.fab[tt[r]] = xi_abar(x[r], (akk[r] > 0.0) - (akk[r] < 0.0));
                            G.fl[tt[r]] = l[r];
                            G.fp[tt[r]] = l[r] == i ? -2 : pp;
                        }
                    }
                }
                fsai_sync<TPR>();
                // denominators of all the group's rows at once, one lane per
                // row, each added in ascending column order
                for (int jj = lane; jj < nk; jj += TPR) {
                    const int off = G.goff[jj], ln = G.goff[jj + 1] - off;
                    double D = 0.0, ai = 0.0;
                    int u = 0;
                    for (; u + 8 <= ln; u += 8) {
                        int pb[8];
                        double xb[8];
#pragma unroll
                        for (int r = 0; r < 8; ++r) {
                            pb[r] = G.fp[off + u + r];
                            xb[r] = G.fab[off + u + r];
                        }
#pragma unroll
                        for (int r = 0; r < 8; ++r) {
                            if (pb[r] >= 0 || (plus_i && pb[r] == -2)) D = D + xb[r];
                            if (pb[r] == -2) ai = xb[r];
                        }
                    }
                    for (; u < ln; ++u) {
                        const int pu = G.fp[off + u];
                        if (pu >= 0 || (plus_i && pu == -2)) D = D + G.fab[off + u];
                        if (pu == -2) ai = G.fab[off + u];
                    }
                    G.gD[jj] = D;
                    G.gai[jj] = ai;
                }
                fsai_sync<TPR>();
                // each set entry adds the shares of the group's rows in CSR
                // order of row i (its column found in each row's sorted
                // columns); rows whose denominator is 0 give none
                for (int pp = lane; pp < U; pp += TPR) {
                    const int col = G.S[pp];
                    double acc = G.num[pp];
                    for (int jj = 0; jj < nk; ++jj) {
                        const double D = G.gD[jj];
                        if (D == 0.0) continue;
                        const int off = G.goff[jj];
                        int lo2 = off, hi2 = G.goff[jj + 1] - 1;
                        while (lo2 <= hi2) {
                            const int mid = lo2 + ((hi2 - lo2) >> 1);
                            const int c2 = G.fl[mid];
                            if (c2 == col) {
                                acc = acc + (G.ma[G.gq[jj]] * G.fab[mid]) / D;
                                break;
                            }
                            if (c2 < col) lo2 = mid + 1;
                            else hi2 = mid - 1;
                        }
                    }
                    G.num[pp] = acc;
                }
                // the diagonal, in CSR order of row i (every lane alike)
                int j = 0;
                for (int t = q; t < qb; ++t) {
                    const int kind = G.mkind[t];
                    const double a = G.ma[t];
                    if (kind == 3) {
                        diag = diag + a;  // weak neighbour outside the set
                    } else if (kind == 1) {
                        const double D = G.gD[j];
                        if (D == 0.0) diag = diag + a;
                        else if (plus_i) diag = diag + (a * G.gai[j]) / D;
                        ++j;
                    }
                }
                fsai_sync<TPR>();
                if (nk == 0 && qb < me) {  // one row longer than CAPF
                    diag = xi_share_long<CAP, CAPF, TPR>(G, i, G.mk[qb], G.ma[qb], G.makk[qb], plus_i, U, diag, rp,
                                                         ci, v, lane);
                    q = qb + 1;
                } else {
                    q = qb;
                }
                fsai_sync<TPR>();
            }
        }
        fsai_sync<TPR>();
        for (int u = lane; u < U; u += TPR) {
            pci[o + u] = (int32_t)cmap[G.S[u]];
            pv[o + u] = -G.num[u] / diag;
        }
    }
}

// ---------------------------------------------------------------- BAMG
// BAMG prolongation (Section 2, Interpolation, eq. minBAMG and Alg. BAMG)
// for a test space V (n x nt, row-major).  The CPU reference's operations in
// its order: each candidate's sums run over the test-space components in
// order, the greedy basis is the largest residual norm with the smallest
// index on ties, and the small sequential steps (projection of phi_i, the
// triangular solve) run on one lane.
constexpr int kBamgNt = 8, kBamgRaw = 1024, kBamgCand = 128;

struct BamgL {
    double l[kBamgNt * kBamgNt];
};

// each row x of V becomes the solution y of L y = x
__global__ void k_ortho_rows(int n, int nt, BamgL L, double *V) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double x[kBamgNt];
    for (int a = 0; a < nt; ++a) x[a] = V[(size_t)r * nt + a];
    for (int a = 0; a < nt; ++a) {
        double t = x[a];
        for (int k = 0; k < a; ++k) t = t - L.l[a * nt + k] * x[k];
        x[a] = t / L.l[a * nt + a];
    }
    for (int a = 0; a < nt; ++a) V[(size_t)r * nt + a] = x[a];
}

struct BamgLds {
    int raw[kBamgRaw], cand[kBamgRaw], first[64];
    int used[kBamgCand];
    double work[kBamgCand * kBamgNt], coef[kBamgCand * kBamgNt];
    double q[kBamgNt * kBamgNt], R[kBamgNt * kBamgNt], w[kBamgNt];
    int sel[kBamgNt];
    int redi[1];
    int cnt, r, best;
    double relres, wn;
};

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, kWave);
        x = y > x ? y : x;
    }
    return x;
}

// Greedy basis and weights of row i over G.cand[0..nc) (one wavefront);
// sets G.r, G.sel, G.w, G.relres, G.wn.
__device__ void bamg_weights(BamgLds &G, int nt, const double *__restrict__ V, int i, int nc, int lane) {
    double n0l = 0.0;
    for (int t = lane; t < nc; t += kWave) {
        G.used[t] = 0;
        double s = 0.0;
        for (int a = 0; a < nt; ++a) {
            const double x = V[(size_t)G.cand[t] * nt + a];
            G.work[t * nt + a] = x;
            s = s + x * x;
        }
        n0l = s > n0l ? s : n0l;
    }
    const double n0 = __longlong_as_double((long long)wave_max_u64((unsigned long long)__double_as_longlong(n0l)));
    FSAI_SYNC();
    int r = 0;
    while (r < nt) {
        // the unused candidate with the largest residual norm, smallest index on ties
        double bl = 0.0;
        int tl = INT_MAX;
        for (int t = lane; t < nc; t += kWave) {
            if (G.used[t]) continue;
            double s = 0.0;
            for (int a = 0; a < nt; ++a) s = s + G.work[t * nt + a] * G.work[t * nt + a];
            if (s > bl) {
                bl = s;
                tl = t;
            }
        }
        const unsigned long long mb = wave_max_u64((unsigned long long)__double_as_longlong(bl));
        const double bn = __longlong_as_double((long long)mb);
        const int best = wave_min_i((unsigned long long)__double_as_longlong(bl) == mb && bl > 0.0 ? tl : INT_MAX);
        if (best == INT_MAX || !(bn > 1e-20 * n0)) break;
        const double nb = sqrt(bn);
        if (lane < nt) G.q[r * kBamgNt + lane] = G.work[best * nt + lane] / nb;
        if (lane < r) G.R[lane * kBamgNt + r] = G.coef[best * nt + lane];
        if (lane == 0) {
            G.R[r * kBamgNt + r] = nb;
            G.used[best] = 1;
            G.sel[r] = best;
        }
        FSAI_SYNC();
        for (int t = lane; t < nc; t += kWave) {
            if (G.used[t]) continue;
            double d = 0.0;
            for (int a = 0; a < nt; ++a) d = d + G.q[r * kBamgNt + a] * G.work[t * nt + a];
            G.coef[t * nt + r] = d;
            for (int a = 0; a < nt; ++a) G.work[t * nt + a] = G.work[t * nt + a] - d * G.q[r * kBamgNt + a];
        }
        FSAI_SYNC();
        ++r;
    }
    if (lane == 0) {
        double res[kBamgNt], c[kBamgNt];
        double ni = 0.0;
        for (int a = 0; a < nt; ++a) {
            res[a] = V[(size_t)i * nt + a];
            ni = ni + res[a] * res[a];
        }
        for (int m = 0; m < r; ++m) {
            double d = 0.0;
            for (int a = 0; a < nt; ++a) d = d + G.q[m * kBamgNt + a] * res[a];
            c[m] = d;
            for (int a = 0; a < nt; ++a) res[a] = res[a] - d * G.q[m * kBamgNt + a];
        }
        for (int m = r - 1; m >= 0; --m) {
            double t = c[m];
            for (int k = m + 1; k < r; ++k) t = t - G.R[m * kBamgNt + k] * G.w[k];
            G.w[m] = t / G.R[m * kBamgNt + m];
        }
        double nr = 0.0, nw = 0.0;
        for (int a = 0; a < nt; ++a) nr = nr + res[a] * res[a];
        for (int m = 0; m < r; ++m) nw = nw + G.w[m] * G.w[m];
        G.relres = ni > 0.0 ? sqrt(nr) / sqrt(ni) : 0.0;
        G.wn = sqrt(nw);
        G.r = r;
    }
    FSAI_SYNC();
}

// One wavefront per row.  C rows: identity.  F rows: candidates at
// distance <= l along strong connections (l <= 2), weights, until the
// relative residual <= eps and ||w|| <= mu or l = lmax.  Row i's entries go
// to tci/tv[i * nt ...], their count to cnt[i].  flags[2]: too many
// candidates.
__global__ void __launch_bounds__(64)
    k_bamg_rows(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                const uint8_t *__restrict__ strong, const int8_t *__restrict__ cf, int nt,
                const double *__restrict__ V, int lmin, int lmax, double eps, double mu,
                const int64_t *__restrict__ cmap, int32_t *cnt, int32_t *tci, double *tv, int32_t *flags) {
    __shared__ BamgLds G;
    const int i = blockIdx.x, lane = threadIdx.x;
    if (i >= n) return;
    if (cf[i] == kC) {
        if (lane == 0) {
            cnt[i] = 1;
            tci[(size_t)i * nt] = (int32_t)cmap[i];
            tv[(size_t)i * nt] = 1.0;
        }
        return;
    }
    const int e0 = rp[i], e1 = rp[i + 1];
    int r = 0, nc = 0;
    double relres = 0.0, wn = 0.0;
    for (int l = lmin; l <= lmax; ++l) {
        if (lane == 0) G.cnt = 0;
        FSAI_SYNC();
        for (int e = e0 + lane; e < e1; e += kWave) {
            const int j = ci[e];
            if (j != i && strong[e] && cf[j] == kC) {
                const int t = atomicAdd(&G.cnt, 1);
                if (t < kBamgRaw) G.raw[t] = j;
            }
        }
        if (l >= 2)
            for (int e = e0; e < e1; ++e) {
                const int j = ci[e];
                if (j == i || !strong[e]) continue;
                for (int f = rp[j] + lane; f < rp[j + 1]; f += kWave) {
                    const int m = ci[f];
                    if (m != j && m != i && strong[f] && cf[m] == kC) {
                        const int t = atomicAdd(&G.cnt, 1);
                        if (t < kBamgRaw) G.raw[t] = m;
                    }
                }
            }
        FSAI_SYNC();
        const int T = G.cnt;
        if (T > kBamgRaw) {
            if (lane == 0) atomicOr(&flags[2], 1);
            return;
        }
        nc = xi_sort_unique<kWave>(G.raw, nullptr, T, G.cand, nullptr, G.first, G.redi, lane);
        if (nc > kBamgCand) {
            if (lane == 0) atomicOr(&flags[2], 1);
            return;
        }
        if (nc > 0) {
            bamg_weights(G, nt, V, i, nc, lane);
            r = G.r;
            relres = G.relres;
            wn = G.wn;
        } else {
            r = 0;
        }
        if (relres <= eps && wn <= mu && r > 0) break;
    }
    if (lane == 0) {
        int ord[kBamgNt];
        for (int m = 0; m < r; ++m) ord[m] = m;
        for (int a = 1; a < r; ++a) {
            const int x = ord[a];
            int b = a - 1;
            while (b >= 0 && G.cand[G.sel[ord[b]]] > G.cand[G.sel[x]]) {
                ord[b + 1] = ord[b];
                --b;
            }
            ord[b + 1] = x;
        }
        for (int m = 0; m < r; ++m) {
            tci[(size_t)i * nt + m] = (int32_t)cmap[G.cand[G.sel[ord[m]]]];
            tv[(size_t)i * nt + m] = G.w[ord[m]];
        }
        cnt[i] = r;
    }
}

// packed rows (nt slots each) -> CSR rows
__global__ void k_bamg_compact(int n, int nt, const int32_t *tci, const double *tv, const int32_t *prp, int32_t *pci,
                               double *pv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int o = prp[i], m = prp[i + 1] - o;
    for (int k = 0; k < m; ++k) {
        pci[o + k] = tci[(size_t)i * nt + k];
        pv[o + k] = tv[(size_t)i * nt + k];
    }
}

// next level's test space: the rows at the C points
__global__ void k_gather_tv(int n, int nt, const int8_t *cf, const int64_t *cmap, const double *V, double *Vc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || cf[i] != kC) return;
    for (int a = 0; a < nt; ++a) Vc[(size_t)cmap[i] * nt + a] = V[(size_t)i * nt + a];
}

// ---------------------------------------------------------------- SRQM
// Test-space refinement by simultaneous Rayleigh quotient minimisation
// (Section 2, near-kernel passage, eq. eigP) with the smoother as
// preconditioner: V <- the nt lowest Ritz vectors of A on span[V, M^{-1} R],
// R = A V - V (V^T A V).  Every sum runs in the CPU reference's order (rows
// of a Gram matrix in index order, the entries of a CSR row in order), so
// the refined space is bitwise the reference's.

constexpr int kSrqmM = 2 * kBamgNt;  // columns of the subspace [V W]

// Y (row stride ldy) = A X (row stride ldx) for k <= 8 columns, one thread per
// (row, column): the k threads of a row share its entries' loads and read
// neighbouring X values, and each sum runs over the row's entries in order
__global__ void k_csr_block(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            const double *__restrict__ v, int k, const double *__restrict__ X, int ldx,
                            double *__restrict__ Y, int ldy) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)n * k) return;
    const int i = (int)(t / k), a = (int)(t % k);
    double acc = 0.0;
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; ++e) acc = acc + v[e] * X[(size_t)ci[e] * ldx + a];
    Y[(size_t)i * ldy + a] = acc;
}

// Gram products G[a * ldg + b] = sum over the rows r = 0..n-1, in order, of
// X[r ldx + a] Y[r ldy + b] (a < ma, b < mb, ma, mb <= 16; only b <= a when
// lower).  The order is fixed, so each sum is one thread's, and the chain of
// n dependent FP64 adds bounds the kernel (about 15 ns per row); the workgroup
// stages 240-row tiles of X and Y in LDS column by column (a padded stride
// keeps 16-byte reads of different columns in different banks), and the
// next tile's loads are in flight while the threads add the current one.
// blockIdx.x selects (Y, G) or (Y2, G2): two products share a launch.
constexpr int kGramRows = 240, kGramThreads = 1024, kGramCols = 16, kGramLd = kGramRows + 2;
constexpr int kGramLoads = (kGramRows * kGramCols + kGramThreads - 1) / kGramThreads;  // per thread and tile

__global__ void __launch_bounds__(kGramThreads)
    k_gram_tiled(int n, int ma, int mb, int lower, const double *__restrict__ X, int ldx, const double *Y,
                 const double *Y2, int ldy, double *G, double *G2, int ldg) {
    __shared__ __align__(16) double xs[kGramCols * kGramLd];
    __shared__ __align__(16) double ys[kGramCols * kGramLd];
    if (blockIdx.x == 1) {
        Y = Y2;
        G = G2;
    }
    const int tid = threadIdx.x;
    int a = -1, b = 0;
    const int npairs = lower ? ma * (ma + 1) / 2 : ma * mb;
    if (tid < npairs) {
        if (lower) {  // pairs (0,0), (1,0), (1,1), (2,0), ...
            int t = tid;
            a = 0;
            while (t > a) {
                t -= a + 1;
                ++a;
            }
            b = t;
        } else {
            a = tid / mb;
            b = tid % mb;
        }
    }
    // this thread's tile elements: row and column within the tile, the same
    // for every tile
    int xr_[kGramLoads], xc_[kGramLoads], yr_[kGramLoads], yc_[kGramLoads];
#pragma unroll
    for (int k = 0; k < kGramLoads; ++k) {
        const int e = tid + k * kGramThreads;
        xr_[k] = e / ma;
        xc_[k] = e % ma;
        yr_[k] = e / mb;
        yc_[k] = e % mb;
    }
    // every thread loads (rows past the matrix are clamped to its last row
    // and not stored), so the loads issue back to back
    double px[kGramLoads], py[kGramLoads];
    auto load = [&](int r0) {
#pragma unroll
        for (int k = 0; k < kGramLoads; ++k) {
            px[k] = X[(size_t)min((int64_t)r0 + xr_[k], (int64_t)n - 1) * ldx + xc_[k]];
            py[k] = Y[(size_t)min((int64_t)r0 + yr_[k], (int64_t)n - 1) * ldy + yc_[k]];
        }
    };
    auto stage = [&](int rows) {
#pragma unroll
        for (int k = 0; k < kGramLoads; ++k) {
            if (xr_[k] < rows) xs[xc_[k] * kGramLd + xr_[k]] = px[k];
            if (yr_[k] < rows) ys[yc_[k] * kGramLd + yr_[k]] = py[k];
        }
    };
    double s = 0.0;
    auto add_tile = [&](int rows) {
        if (a < 0) return;
        // 16 rows' products are formed first (independent of each other, two
        // rows per 16-byte read), then added in row order
        const double *xr = xs + a * kGramLd, *yr = ys + b * kGramLd;
        const double2 *x2 = reinterpret_cast<const double2 *>(xr);
        const double2 *y2 = reinterpret_cast<const double2 *>(yr);
        int r = 0;
        for (; r + 16 <= rows; r += 16) {
            double pv[16];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double2 xv = x2[(r >> 1) + u], yv = y2[(r >> 1) + u];
                pv[2 * u] = xv.x * yv.x;
                pv[2 * u + 1] = xv.y * yv.y;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) s = s + pv[u];
        }
        for (; r < rows; ++r) s = s + xr[r] * yr[r];
    };
    if (n > 0) load(0);
    for (int r0 = 0; r0 < n; r0 += kGramRows) {
        const int rows = min(kGramRows, n - r0);
        stage(rows);
        __syncthreads();
        if (r0 + kGramRows < n) load(r0 + kGramRows);
        add_tile(rows);
        __syncthreads();
    }
    if (a >= 0) G[a * ldg + b] = s;
}

// R = X - V T per row (V, X: the first nt columns of S and AS, stride m);
// out (stride ldo) = dinv[r] R (Jacobi) or R (dinv null)
__global__ void k_srqm_resid(int n, int nt, int m, const double *__restrict__ S, const double *__restrict__ AS,
                             const double *__restrict__ T, const double *__restrict__ dinv, double *__restrict__ out,
                             int ldo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double vr[kBamgNt];
#pragma unroll
    for (int a = 0; a < kBamgNt; ++a) vr[a] = a < nt ? S[(size_t)i * m + a] : 0.0;
    const double d = dinv ? dinv[i] : 1.0;
#pragma unroll
    for (int b = 0; b < kBamgNt; ++b) {
        if (b >= nt) break;
        double r = AS[(size_t)i * m + b];
#pragma unroll
        for (int a = 0; a < kBamgNt; ++a)
            if (a < nt) r = r - vr[a] * T[a * nt + b];
        out[(size_t)i * ldo + b] = dinv ? d * r : r;
    }
}

// The Rayleigh-Ritz step on the Gram matrices Gs = S^T S and Hs = S^T A S
// (lower triangles, m = 2 nt), one wavefront:
//   up-looking Cholesky of Gs leaving out columns with pivot <= 1e-12 of the
//   largest diagonal (lane 0); C = L^{-1} Hs L^{-T} (a lane per column);
//   cyclic Jacobi on C (a lane per row / column of each rotation); the nt
//   smallest eigenvalues (smaller index on ties) and Z = L^{-T} Q_sel (a lane
//   per column).  Out: kept columns K[0..mk), Z (mk x nt), mk (*mko).
__global__ void __launch_bounds__(kWave) k_srqm_rr(int nt, const double *__restrict__ Gs,
                                                   const double *__restrict__ Hs, int32_t *__restrict__ Ko,
                                                   double *__restrict__ Zo, int32_t *__restrict__ mko) {
    constexpr int M = kSrqmM;
    __shared__ double g[M * M], h[M * M], L[M * M], Cm[M * M], C[M * M], Q[M * M], lam[M];
    __shared__ int K[M], sel[kBamgNt];
    __shared__ int mk_s, go;
    __shared__ double tot_s;
    const int lane = threadIdx.x;
    const int m = 2 * nt;
    for (int t = lane; t < m * m; t += kWave) {
        const int a = t / m, b = t % m;
        const int lo = a >= b ? a * m + b : b * m + a;  // the lower-triangle entry
        g[t] = Gs[lo];
        h[t] = Hs[lo];
    }
    __syncthreads();
    if (lane == 0) {
        double gmax = 0.0;
        for (int a = 0; a < m; ++a) gmax = g[a * m + a] > gmax ? g[a * m + a] : gmax;
        int mk = 0;
        for (int j = 0; j < m; ++j) {
            for (int k = 0; k < mk; ++k) {
                double t = g[j * m + K[k]];
                for (int q = 0; q < k; ++q) t = t - L[mk * M + q] * L[k * M + q];
                L[mk * M + k] = t / L[k * M + k];
            }
            double d = g[j * m + j];
            for (int k = 0; k < mk; ++k) d = d - L[mk * M + k] * L[mk * M + k];
            if (!(d > 1e-12 * gmax)) continue;
            L[mk * M + mk] = sqrt(d);
            K[mk] = j;
            ++mk;
        }
        mk_s = mk;
        *mko = mk;
        for (int k = 0; k < mk; ++k) Ko[k] = K[k];
    }
    __syncthreads();
    const int mk = mk_s;
    if (mk <= nt) return;  // W adds no direction: the caller stops
    // Cm = L^{-1} H' (H' = Hs on the kept columns), one column per lane
    if (lane < mk) {
        const int c = lane;
        for (int r = 0; r < mk; ++r) {
            double t = h[K[r] * m + K[c]];
            for (int q = 0; q < r; ++q) t = t - L[r * M + q] * Cm[q * M + c];
            Cm[r * M + c] = t / L[r * M + r];
        }
    }
    __syncthreads();
    // Q = L^{-1} Cm^T (temporary), one column per lane
    if (lane < mk) {
        const int c = lane;
        for (int r = 0; r < mk; ++r) {
            double t = Cm[c * M + r];
            for (int q = 0; q < r; ++q) t = t - L[r * M + q] * Q[q * M + c];
            Q[r * M + c] = t / L[r * M + r];
        }
    }
    __syncthreads();
    for (int t = lane; t < mk * mk; t += kWave) {
        const int r = t / mk, c = t % mk;
        C[r * M + c] = r >= c ? Q[r * M + c] : Q[c * M + r];
    }
    __syncthreads();
    for (int t = lane; t < mk * mk; t += kWave) {
        const int r = t / mk, c = t % mk;
        Q[r * M + c] = r == c ? 1.0 : 0.0;
    }
    if (lane == 0) {
        double tot = 0.0;
        for (int i = 0; i < mk; ++i)
            for (int j = 0; j < mk; ++j) tot = tot + C[i * M + j] * C[i * M + j];
        tot_s = tot;
    }
    __syncthreads();
    // cyclic Jacobi (Golub and Van Loan's symmetric Schur rotation)
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (lane == 0) {
            double off = 0.0;
            for (int p = 0; p < mk; ++p)
                for (int q = p + 1; q < mk; ++q) off = off + C[p * M + q] * C[p * M + q];
            go = off > 1e-30 * tot_s;
        }
        __syncthreads();
        if (!go) break;
        for (int p = 0; p < mk; ++p)
            for (int q = p + 1; q < mk; ++q) {
                const double apq = C[p * M + q];
                if (apq == 0.0) continue;  // uniform: every lane reads the same value
                const double tau = (C[q * M + q] - C[p * M + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                __syncthreads();
                if (lane < mk) {
                    const int k = lane;
                    const double x = C[k * M + p], y = C[k * M + q];
                    C[k * M + p] = c * x - s * y;
                    C[k * M + q] = s * x + c * y;
                }
                __syncthreads();
                if (lane < mk) {
                    const int k = lane;
                    const double x = C[p * M + k], y = C[q * M + k];
                    C[p * M + k] = c * x - s * y;
                    C[q * M + k] = s * x + c * y;
                    const double u = Q[k * M + p], w = Q[k * M + q];
                    Q[k * M + p] = c * u - s * w;
                    Q[k * M + q] = s * u + c * w;
                }
                __syncthreads();
            }
    }
    if (lane == 0) {
        for (int i = 0; i < mk; ++i) lam[i] = C[i * M + i];
        bool used[M];
        for (int k = 0; k < mk; ++k) used[k] = false;
        for (int b = 0; b < nt; ++b) {
            int best = -1;
            for (int k = 0; k < mk; ++k)
                if (!used[k] && (best < 0 || lam[k] < lam[best])) best = k;
            used[best] = true;
            sel[b] = best;
        }
    }
    __syncthreads();
    // Z = L^{-T} Q_sel, one column per lane (back substitution)
    if (lane < nt) {
        const int b = lane, best = sel[b];
        double z[M];
        for (int r = mk - 1; r >= 0; --r) {
            double t = Q[r * M + best];
            for (int q = r + 1; q < mk; ++q) t = t - L[q * M + r] * z[q];
            z[r] = t / L[r * M + r];
        }
        for (int r = 0; r < mk; ++r) Zo[r * nt + b] = z[r];
    }
}

// V = S_kept Z per row, written over the first nt columns of S
__global__ void k_srqm_combine(int n, int nt, int m, const int32_t *__restrict__ K, const int32_t *__restrict__ mkp,
                               const double *__restrict__ Z, double *__restrict__ S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int mk = *mkp;
    double row[kSrqmM];
#pragma unroll
    for (int k = 0; k < kSrqmM; ++k) row[k] = k < mk ? S[(size_t)i * m + K[k]] : 0.0;
#pragma unroll
    for (int b = 0; b < kBamgNt; ++b) {
        if (b >= nt) break;
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < kSrqmM; ++k)
            if (k < mk) t = t + row[k] * Z[k * nt + b];
        S[(size_t)i * m + b] = t;
    }
}

// Y (stride ldy, k columns) = X (stride ldx)
__global__ void k_copy_block(int n, int k, const double *__restrict__ X, int ldx, double *__restrict__ Y, int ldy) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)n * k) return;
    const size_t r = t / k, a = t % k;
    Y[r * ldy + a] = X[r * ldx + a];
}

// ---------------------------------------------------------------- P smoothing and filtering
// Ps = P - omega D^{-1} (A P): one thread per row merges the rows of P and
// A P (entry p - (omega dinv_i) ap, a missing entry read as 0).
template <bool FILL>
__global__ void k_psmooth(int n, const int32_t *prp, const int32_t *pci, const double *pv, const int32_t *arp,
                          const int32_t *aci, const double *av, const double *dinv, double omega, int32_t *cnt,
                          const int32_t *srp, int32_t *sci, double *sv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = prp[i], b = arp[i];
    const int a1 = prp[i + 1], b1 = arp[i + 1];
    const double sc = omega * dinv[i];
    int o = FILL ? srp[i] : 0, c = 0;
    while (a < a1 || b < b1) {
        const int ja = a < a1 ? pci[a] : INT_MAX, jb = b < b1 ? aci[b] : INT_MAX;
        const int j = ja < jb ? ja : jb;
        double p = 0.0, q = 0.0;
        if (ja == j) p = pv[a++];
        if (jb == j) q = av[b++];
        if (FILL) {
            sci[o + c] = j;
            sv[o + c] = p - sc * q;
        }
        ++c;
    }
    if (!FILL) cnt[i] = c;
}

// Filtering with compensation: one wavefront per row.  The entries are
// ranked by decreasing |p| (smaller column first on ties) in LDS; lane 0
// finds the kept prefix (absolute values added in rank order); the
// dropped action r on W and the Gram matrix of the kept rows of W are sums
// in ascending column order (one lane per component or pair); lane 0
// solves (B B^T + lambda I) y = r; kept entries become p + W_k . y.
constexpr int kFiltMax = 1024;

__global__ void __launch_bounds__(64) k_pfilter(int n, const int32_t *rp, const int32_t *ci, const double *v, double rho,
                                                int nt, const double *W, int32_t *cnt, int32_t *tci, double *tvv,
                                                int32_t *flags) {
    __shared__ int rk[kFiltMax];
    __shared__ unsigned char keep[kFiltMax];
    __shared__ double r[kBamgNt], G[kBamgNt * kBamgNt], y[kBamgNt];
    __shared__ int dropped;
    const int i = blockIdx.x, lane = threadIdx.x;
    if (i >= n) return;
    const int e0 = rp[i], m = rp[i + 1] - e0;
    if (m > kFiltMax) {
        if (lane == 0) atomicOr(&flags[2], 1);
        return;
    }
    for (int t = lane; t < m; t += kWave) keep[t] = 1;
    if (lane == 0) dropped = 0;
    FSAI_SYNC();
    if (rho < 1.0 && m > 1) {
        // rank of each entry in the (|p| desc, column asc) order
        for (int t = lane; t < m; t += kWave) {
            const double x = fabs(v[e0 + t]);
            const int c = ci[e0 + t];
            int k = 0;
            for (int u = 0; u < m; ++u) {
                const double yv = fabs(v[e0 + u]);
                const int cu = ci[e0 + u];
                k += (yv > x || (yv == x && cu < c)) ? 1 : 0;
            }
            rk[k] = t;
        }
        FSAI_SYNC();
        if (lane == 0) {
            double tot = 0.0, run = 0.0;
            for (int k = 0; k < m; ++k) tot = tot + fabs(v[e0 + rk[k]]);
            int nk = 0;
            while (nk < m && run < rho * tot) run = run + fabs(v[e0 + rk[nk++]]);
            if (nk < 1) nk = 1;
            for (int t = 0; t < m; ++t) keep[t] = 0;
            for (int k = 0; k < nk; ++k) keep[rk[k]] = 1;
            dropped = nk < m ? 1 : 0;
        }
        FSAI_SYNC();
    }
    const int drop = dropped;
    if (drop) {
        if (lane < nt) {
            double ra = 0.0;
            for (int t = 0; t < m; ++t)
                if (!keep[t]) ra = ra + v[e0 + t] * W[(size_t)ci[e0 + t] * nt + lane];
            r[lane] = ra;
        }
        for (int pq = lane; pq < nt * nt; pq += kWave) {
            const int a = pq / nt, b = pq % nt;
            if (b > a) continue;
            double g = 0.0;
            for (int t = 0; t < m; ++t)
                if (keep[t]) g = g + W[(size_t)ci[e0 + t] * nt + a] * W[(size_t)ci[e0 + t] * nt + b];
            G[a * nt + b] = g;
        }
        FSAI_SYNC();
        if (lane == 0) {
            double tr = 0.0;
            for (int a = 0; a < nt; ++a) tr = tr + G[a * nt + a];
            const double lam = 1e-12 * tr / nt;
            for (int a = 0; a < nt; ++a) G[a * nt + a] = G[a * nt + a] + lam;
            for (int j = 0; j < nt; ++j) {
                double d = G[j * nt + j];
                for (int k = 0; k < j; ++k) d = d - G[j * nt + k] * G[j * nt + k];
                const double ljj = sqrt(d > 0.0 ? d : 0.0);
                G[j * nt + j] = ljj;
                for (int q = j + 1; q < nt; ++q) {
                    double t = G[q * nt + j];
                    for (int k = 0; k < j; ++k) t = t - G[q * nt + k] * G[j * nt + k];
                    G[q * nt + j] = ljj > 0.0 ? t / ljj : 0.0;
                }
            }
            for (int a = 0; a < nt; ++a) {
                double t = r[a];
                for (int k = 0; k < a; ++k) t = t - G[a * nt + k] * y[k];
                y[a] = G[a * nt + a] > 0.0 ? t / G[a * nt + a] : 0.0;
            }
            for (int a = nt - 1; a >= 0; --a) {
                double t = y[a];
                for (int k = a + 1; k < nt; ++k) t = t - G[k * nt + a] * y[k];
                y[a] = G[a * nt + a] > 0.0 ? t / G[a * nt + a] : 0.0;
            }
        }
        FSAI_SYNC();
    }
    // kept entries in ascending column order (their position: kept before them)
    for (int t = lane; t < m; t += kWave) {
        if (!keep[t]) continue;
        int pos = 0;
        for (int u = 0; u < t; ++u) pos += keep[u];
        double d = 0.0;
        if (drop)
            for (int a = 0; a < nt; ++a) d = d + W[(size_t)ci[e0 + t] * nt + a] * y[a];
        tci[e0 + pos] = ci[e0 + t];
        tvv[e0 + pos] = v[e0 + t] + d;
    }
    if (lane == 0) {
        int k = 0;
        for (int t = 0; t < m; ++t) k += keep[t];
        cnt[i] = k;
    }
}

// rows of a temporary laid out like the source (row i at src_rp[i]) -> CSR
__global__ void k_compact_rows(int n, const int32_t *src_rp, const int32_t *tci, const double *tv, const int32_t *rp,
                               int32_t *ci, double *v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s0 = src_rp[i], o = rp[i], m = rp[i + 1] - o;
    for (int k = 0; k < m; ++k) {
        ci[o + k] = tci[s0 + k];
        v[o + k] = tv[s0 + k];
    }
}

__global__ void k_fill_ones(int n, double *x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 1.0;
}

// Relaxation weight of the FSAI smoother (eq. smoother, eq. smo): the
// Rayleigh quotient of M = G A G^T after kFsaiPowerSteps power steps, M
// applied as G (A (G^T v)).  Start: v_i = 2 u_i - 1, u_i the top 53 bits of
// splitmix64 draw ((level << 40) + i) of a generator seeded with seed + 1,
// over 2^53.  Products summed in CSR order from 0.0 (the oracle's order);
// the dot products by a fixed tree.
constexpr int kFsaiPowerSteps = 15;
constexpr int kPwGrid = 1024;  // blocks of the dot-product kernel (partials per dot)

__global__ void k_pw_start(int n, uint64_t seed, int level, double *v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint64_t c = ((uint64_t)(uint32_t)level << 40) + (uint64_t)(uint32_t)i;
        v[i] = 2.0 * ((double)(splitmix64(seed + 1u, c) >> 11) * 0x1p-53) - 1.0;
    }
}

// y = M x with G lanes per row: the lanes form G products at a time, which
// every lane then adds in CSR order (the sum a thread walking the row forms)
template <int G>
__global__ void __launch_bounds__(kBlock) k_pw_spmv(int n, const int32_t *rp, const int32_t *ci, const double *mv,
                                                    const double *x, double *y) {
    int sl;
    const int i = group_row<G>(n, sl);
    const int e0 = i < n ? rp[i] : 0, e1 = i < n ? rp[i + 1] : 0;
    double s = 0.0;
    for (int c = e0; c < e1; c += G) {
        const int e = c + sl;
        const double p = e < e1 ? mv[e] * x[ci[e]] : 0.0;
        const int cnt = min(G, e1 - c);
        for (int k = 0; k < cnt; ++k) s = s + __shfl(p, k, G);
    }
    if (i < n && sl == 0) y[i] = s;
}

// partials of v.v, v.w, w.w (block b: part[3 b + 0..2])
__global__ void __launch_bounds__(kBlock) k_pw_dots(int n, const double *v, const double *w, double *part) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        a = a + v[i] * v[i];
        b = b + v[i] * w[i];
        c = c + w[i] * w[i];
    }
    a = block_sum<kBlock>(a);
    b = block_sum<kBlock>(b);
    c = block_sum<kBlock>(c);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = c;
    }
}

// st[0] = v.w / v.v (the Rayleigh quotient), st[1] = 1 / ||w||
__global__ void __launch_bounds__(kBlock) k_pw_fin(int nb, const double *part, double *st) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int t = threadIdx.x; t < nb; t += kBlock) {
        a = a + part[3 * t];
        b = b + part[3 * t + 1];
        c = c + part[3 * t + 2];
    }
    a = block_sum<kBlock>(a);
    b = block_sum<kBlock>(b);
    c = block_sum<kBlock>(c);
    if (threadIdx.x == 0) {
        st[0] = b / a;
        st[1] = 1.0 / sqrt(c);
    }
}

__global__ void k_pw_scale(int n, const double *w, const double *st, double *v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = w[i] * st[1];
}

__global__ void k_fill_d(int n, double *v, double x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = x;
}

__global__ void k_max_row(int n, const int32_t *rp, int32_t *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int len = i < n ? rp[i + 1] - rp[i] : 0;
    const unsigned long long m = block_max_u64<kBlock>((unsigned long long)len);
    if (threadIdx.x == 0) fold_max(out, (int32_t)m);
}

// Tiles of the row kernels: tile t holds the rows whose first nonzero lies
// in [t W, (t+1) W).  tstart[t] = first row of tile t; tstart[ntiles] = n.
__global__ void k_tile_starts(int n, const int32_t *rp, int W, int ntiles, int32_t *tstart) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        const int tp = rp[n - 1] / W;
        for (int t = tp + 1; t <= ntiles; ++t) tstart[t] = n;
        return;
    }
    const int ti = rp[i] / W;
    const int tp = i == 0 ? -1 : rp[i - 1] / W;
    for (int t = tp + 1; t <= ti && t < ntiles; ++t) tstart[t] = i;
}


// Compact column indices of a tiled matrix: tile t keeps up to kTileWins
// windows of 2^kWinBits columns, chosen greedily (window w starts at the
// smallest column at or past the end of window w - 1), in tbase[t * kTileWins
// ...]; a nonzero stores its window in the top bits of a 16-bit word and its
// offset in the window in the low kWinBits bits.  When every tile spans fewer
// than 65536 columns the words are simply column - (first window start), and
// the kernels need no window table.  One block per tile: k_tile_bases places
// the windows (unused slots repeat the last one), sets flag[0] when the tile
// needs more and flag[1] when it spans 65536 columns or more; k_tile_diffs
// writes the 16-bit words (single = 1: plain differences).
__global__ void __launch_bounds__(kBlock) k_tile_bases(int ntiles, const int32_t *__restrict__ tstart,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, int32_t *tbase,
                                                       int32_t *flag) {
    __shared__ int next_s;
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const int e0 = rp[tstart[t]], e1 = rp[tstart[t + 1]];
    {  // one 65536-column span from the smallest column?
        int lo = INT32_MAX, hi = 0;
        for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) {
            lo = min(lo, ci[e]);
            hi = max(hi, ci[e]);
        }
        const unsigned long long mlo = block_max_u64<kBlock>((unsigned long long)(INT32_MAX - lo));
        const unsigned long long mhi = block_max_u64<kBlock>((unsigned long long)hi);
        if (threadIdx.x == 0 && e1 > e0 && (int)mhi - (INT32_MAX - (int)mlo) > 65535) flag[1] = 1;
    }
    int from = 0, last = 0;
    for (int w = 0; w < kTileWins; ++w) {
        int lo = INT32_MAX;
        for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock)
            if (ci[e] >= from) lo = min(lo, ci[e]);
        const unsigned long long m = block_max_u64<kBlock>((unsigned long long)(INT32_MAX - lo));
        if (threadIdx.x == 0) next_s = INT32_MAX - (int)m;
        __syncthreads();
        const int start = next_s;
        __syncthreads();
        if (start == INT32_MAX) {  // every column is covered
            for (int v = w + (int)threadIdx.x; v < kTileWins; v += kBlock) tbase[t * kTileWins + v] = last;
            return;
        }
        if (threadIdx.x == 0) tbase[t * kTileWins + w] = start;
        last = start;
        from = start > INT32_MAX - (1 << kWinBits) ? INT32_MAX : start + (1 << kWinBits);
    }
    // columns past the last window: the tile needs more windows
    int over = 0;
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) over |= ci[e] >= from;
    const unsigned long long any = block_max_u64<kBlock>((unsigned long long)over);
    if (threadIdx.x == 0 && any) {
        flag[0] = 1;
        flag[1] = 1;
    }
}

__global__ void __launch_bounds__(kBlock) k_tile_diffs(int ntiles, const int32_t *__restrict__ tstart,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const int32_t *__restrict__ tbase, uint16_t *off, int single) {
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const int e0 = rp[tstart[t]], e1 = rp[tstart[t + 1]];
    int w[kTileWins];
#pragma unroll
    for (int v = 0; v < kTileWins; ++v) w[v] = tbase[t * kTileWins + v];
    if (single) {
        for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) off[e] = (uint16_t)(ci[e] - w[0]);
        return;
    }
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kBlock) {
        const int c = ci[e];
        int slot = 0, base = w[0];
#pragma unroll
        for (int v = 1; v < kTileWins; ++v)
            if (c >= w[v] && w[v] > w[v - 1]) {
                slot = v;
                base = w[v];
            }
        off[e] = (uint16_t)((slot << kWinBits) | (c - base));
    }
}
}  // namespace

// ---------------------------------------------------------------- launchers
void scan_i32_to_i64(const int32_t *in, int64_t *out, int n, Pool &tmp, hipStream_t s) { scan_impl(in, out, n, tmp, s); }
void scan_i64(const int64_t *in, int64_t *out, int n, Pool &tmp, hipStream_t s) { scan_impl(in, out, n, tmp, s); }
void narrow_i64(const int64_t *v, int32_t *o, int n, hipStream_t s) {
    k_narrow<<<nblocks(n + 1), kBlock, 0, s>>>(v, o, n);
    HIPC(hipGetLastError());
}

void validate_rowptr(int n, int64_t nnz, const int32_t *rp, int32_t *flags, hipStream_t s) {
    k_val_rowptr<<<nblocks(n), kBlock, 0, s>>>(n, nnz, rp, flags);
    HIPC(hipGetLastError());
}
void validate_rows(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, int32_t *flags,
                   unsigned long long *amax, hipStream_t s) {
    const int g = group_lanes(n, nnz);
    CAMG_G_SWITCH(g, (k_val_rows_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, v, flags, amax)));
    HIPC(hipGetLastError());
}
void validate_sym(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v,
                  const unsigned long long *amax, int32_t *flags, int32_t *tpos, hipStream_t s) {
    const int g = group_lanes(n, nnz);
    CAMG_G_SWITCH(g, (k_tpos_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, v, amax, flags, tpos)));
    HIPC(hipGetLastError());
}
void transpose_positions(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, int32_t *tpos, hipStream_t s) {
    const int g = group_lanes(n, nnz);
    CAMG_G_SWITCH(g, (k_tpos_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, nullptr, nullptr, nullptr, tpos)));
    HIPC(hipGetLastError());
}
void strength(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *tpos,
              double theta, uint8_t *strong, int32_t *stcnt, hipStream_t s) {
    const int g = group_lanes(n, nnz);
    CAMG_G_SWITCH(g, (k_strength_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, v, theta, strong)));
    CAMG_G_SWITCH(g, (k_stcount_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, tpos, strong, stcnt)));
    HIPC(hipGetLastError());
}
void pmis_init(int n, const int32_t *stcnt, uint64_t seed, int level, uint64_t *u, int8_t *state,
               int32_t *undecided, hipStream_t s) {
    HIPC(hipMemsetAsync(undecided, 0, sizeof(int32_t), s));
    k_pmis_init<<<nblocks(n), kBlock, 0, s>>>(n, stcnt, seed, level, u, state, undecided);
    HIPC(hipGetLastError());
}
// Lanes per row of a PMIS round: about eight entries per lane.  Most rows
// are decided after the first rounds and leave at once, so wider groups
// mostly add wavefronts that do nothing (measured on strength + PMIS: one
// lane per entry took 1.6x as long on 7-point rows, one lane per row 1.7x
// as long on 81-entry rows).
inline int pmis_lanes(int n, int64_t nnz) { return std::max(1, group_lanes(n, nnz) / 8); }
void pmis_round(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const uint8_t *strong,
                const int32_t *tpos, const int32_t *stcnt, const uint64_t *u, int8_t *state, int8_t *newc,
                int32_t *undecided, hipStream_t s) {
    const int g = pmis_lanes(n, nnz);
    CAMG_G_SWITCH(g, (k_pmis_select_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, strong, tpos, stcnt, u,
                                                                                 state, newc)));
    HIPC(hipMemsetAsync(undecided, 0, sizeof(int32_t), s));
    CAMG_G_SWITCH(g, (k_pmis_update_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, strong, newc, state,
                                                                                 undecided)));
    HIPC(hipGetLastError());
}
void cf_flags(int n, const int8_t *cf, int32_t *isc, hipStream_t s) {
    k_cf_flags<<<nblocks(n), kBlock, 0, s>>>(n, cf, isc);
    HIPC(hipGetLastError());
}
void interp_count(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const uint8_t *strong,
                  const int8_t *cf, int32_t *cnt, hipStream_t s) {
    const int g = group_lanes(n, nnz);
    CAMG_G_SWITCH(g, (k_interp_count_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, strong, cf, cnt)));
    HIPC(hipGetLastError());
}
void interp_fill(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, const uint8_t *strong,
                 const int8_t *cf, const int64_t *cmap, const int32_t *prp, int32_t *pci, double *pv, hipStream_t s) {
    // three ordered sums as long as the row whatever G is (see diag_gershgorin)
    const int g = std::min(group_lanes(n, nnz), kOrderedLanes);
    CAMG_G_SWITCH(g, (k_interp_fill_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, v, strong, cf, cmap, prp,
                                                                                 pci, pv)));
    HIPC(hipGetLastError());
}
void column_counts(const Csr &X, int32_t *cnt, hipStream_t s) {
    HIPC(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)X.nc, s));
    if (X.nnz > 0) k_col_count<<<nblocks(X.nnz), kBlock, 0, s>>>(X.nnz, X.ci, cnt);
    HIPC(hipGetLastError());
}
void transpose_csr(const Csr &X, Csr &XT, Pool &tmp, hipStream_t s) {
    // XT.rp must already hold the row pointer (from column_counts + scan)
    int32_t *fill = tmp.alloc<int32_t>((size_t)X.nc + 1);
    HIPC(hipMemcpyAsync(fill, XT.rp, sizeof(int32_t) * ((size_t)X.nc + 1), hipMemcpyDeviceToDevice, s));
    k_transpose_fill<<<nblocks(X.nr), kBlock, 0, s>>>(X.nr, X.rp, X.ci, X.v, fill, XT.ci, XT.v);
    HIPC(hipGetLastError());
    const int nc = X.nc;
    int32_t *list = tmp.alloc<int32_t>(std::max(nc, 1)), *cnt = tmp.alloc<int32_t>(1);
    HIPC(hipMemsetAsync(cnt, 0, sizeof(int32_t), s));
    k_long_rows<<<nblocks(nc), kBlock, 0, s>>>(nc, XT.rp, kSortWave, list, cnt);
    HIPC(hipGetLastError());
    int32_t nlong = 0;
    HIPC(hipMemcpyAsync(&nlong, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (nlong > 0) {
        int32_t *sci = tmp.alloc<int32_t>(padded(X.nnz));
        double *sv = tmp.alloc<double>(padded(X.nnz));
        HIPC(hipMemcpyAsync(sci, XT.ci, sizeof(int32_t) * X.nnz, hipMemcpyDeviceToDevice, s));
        HIPC(hipMemcpyAsync(sv, XT.v, sizeof(double) * X.nnz, hipMemcpyDeviceToDevice, s));
        k_sort_rows_block<<<nlong, 1024, 0, s>>>(list, XT.rp, sci, sv, XT.ci, XT.v);
    }
    const int smax = nc >= kSortThreadRows ? kSortShort : 1;
    if (smax > 1) k_sort_rows<<<nblocks(nc), kBlock, 0, s>>>(nc, XT.rp, XT.ci, XT.v, smax);
    k_sort_rows_wave<<<(nc + 3) / 4, 256, 0, s>>>(nc, XT.rp, XT.ci, XT.v, smax);
    HIPC(hipGetLastError());
}
void diag_gershgorin(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, double *dinv,
                     unsigned long long *qmax, int32_t *flags, hipStream_t s) {
    HIPC(hipMemsetAsync(qmax, 0, sizeof(unsigned long long), s));
    // the ordered sum is a chain as long as the row whatever G is, so fewer
    // lanes per row keep more rows in flight per wavefront
    const int g = std::min(group_lanes(n, nnz), kOrderedLanes);
    CAMG_G_SWITCH(g, (k_diag_gersh_g<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, rp, ci, v, dinv, qmax, flags)));
    HIPC(hipGetLastError());
}
void scale_vec(int n, double omega, const double *dinv, double *wd, hipStream_t s) {
    k_scale<<<nblocks(n), kBlock, 0, s>>>(n, omega, dinv, wd);
    HIPC(hipGetLastError());
}
void scale_columns(const Csr &A, const double *wd, double *awd, hipStream_t s) {
    if (A.nnz > 0)
        k_scale_entries<<<(int)((A.nnz + kBlock - 1) / kBlock), kBlock, 0, s>>>(A.nnz, A.ci, A.v, wd, awd);
    HIPC(hipGetLastError());
}

void to_f32(int64_t n, const double *in, float *out, hipStream_t s) {
    if (n > 0) k_to_f32<<<nblocks(n), kBlock, 0, s>>>(n, in, out);
    HIPC(hipGetLastError());
}
void dense_from_csr(int n, const int32_t *rp, const int32_t *ci, const double *v, double *D, hipStream_t s) {
    const int64_t nn = (int64_t)n * n;
    k_dense_zero<<<nblocks(nn), kBlock, 0, s>>>(nn, D);
    k_dense_from_csr<<<nblocks(n), kBlock, 0, s>>>(n, rp, ci, v, D);
    HIPC(hipGetLastError());
}
void cholesky_dense(int n, double *D, int32_t *flags, hipStream_t s) {
    if (n <= kCholMfmaMax) k_cholesky_mfma<<<1, 512, 0, s>>>(n, D, flags);
    else k_cholesky<<<1, 1024, 0, s>>>(n, D, flags);
    HIPC(hipGetLastError());
}
void chol_inverse(int n, const double *L, double *X, hipStream_t s) {
    k_chol_inverse<<<n, 64, sizeof(double) * (size_t)n, s>>>(n, L, X);
    HIPC(hipGetLastError());
}
void tile_starts(int n, const int32_t *rp, int W, int ntiles, int32_t *tstart, hipStream_t s) {
    k_tile_starts<<<nblocks(n + 1), kBlock, 0, s>>>(n, rp, W, ntiles, tstart);
    HIPC(hipGetLastError());
}

void max_row_length_async(int n, const int32_t *rp, int32_t *out, hipStream_t s) {
    k_max_row<<<nblocks(n), kBlock, 0, s>>>(n, rp, out);
    HIPC(hipGetLastError());
}

void tile_bases_async(int ntiles, const int32_t *tstart, const int32_t *rp, const int32_t *ci, int32_t *tbase,
                      int32_t *flag, hipStream_t s) {
    if (ntiles > 0) k_tile_bases<<<ntiles, kBlock, 0, s>>>(ntiles, tstart, rp, ci, tbase, flag);
    HIPC(hipGetLastError());
}

void tile_diffs(int ntiles, const int32_t *tstart, const int32_t *rp, const int32_t *ci, const int32_t *tbase,
                uint16_t *off, int mode, hipStream_t s) {
    k_tile_diffs<<<ntiles, kBlock, 0, s>>>(ntiles, tstart, rp, ci, tbase, off, mode == 1);
    HIPC(hipGetLastError());
}


int fsai_counts(int n, const int32_t *rp, const int32_t *ci, int32_t *cnt, Pool &tmp, hipStream_t s) {
    int32_t *d = tmp.alloc<int32_t>(1);
    HIPC(hipMemsetAsync(d, 0, sizeof(int32_t), s));
    k_fsai_count<<<nblocks(n), kBlock, 0, s>>>(n, rp, ci, cnt, d);
    HIPC(hipGetLastError());
    int32_t h = 0;
    HIPC(hipMemcpyAsync(&h, d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    return h;
}

void fsai_rows(const Csr &A, Csr &G, int mmax, int32_t *flags, hipStream_t s) {
    const int n = A.nr;
    if (mmax <= 16) k_fsai_rows<16, 4, 64><<<(n + 3) / 4, 256, 0, s>>>(n, A.rp, A.ci, A.v, G.rp, G.ci, G.v, flags);
    else if (mmax <= 32) k_fsai_rows<32, 4, 64><<<(n + 3) / 4, 256, 0, s>>>(n, A.rp, A.ci, A.v, G.rp, G.ci, G.v, flags);
    else if (mmax <= 64) k_fsai_rows<64, 1, 64><<<n, 64, 0, s>>>(n, A.rp, A.ci, A.v, G.rp, G.ci, G.v, flags);
    else if (mmax <= 128) k_fsai_rows<128, 1, 256><<<n, 256, 0, s>>>(n, A.rp, A.ci, A.v, G.rp, G.ci, G.v, flags);
    else if (mmax <= kFsaiMaxRow) k_fsai_rows<kFsaiMaxRow, 1, 256><<<n, 256, 0, s>>>(n, A.rp, A.ci, A.v, G.rp, G.ci, G.v, flags);
    else fail(CAMG_E_ARG, "FSAI: a row has more than 192 entries on or below the diagonal");
    HIPC(hipGetLastError());
}

void afsai_rows(const Csr &A, const int32_t *tpos, int maxrow, int steps, int step, double eps, int32_t *cnt,
                int32_t *pci, double *pv, int32_t *flags, hipStream_t s) {
    const int n = A.nr;
    const int mcap = steps * step + 1;
    if (steps < 0 || step < 1 || mcap > kAfsaiMaxM) fail(CAMG_E_ARG, "aFSAI: steps * step + 1 must be at most 32");
    const int64_t bound = (int64_t)mcap * std::max(maxrow, 1);  // candidates of a row never exceed this
#define AFSAI_LAUNCH(MM, CAP, WPB)                                                                            \
    k_afsai_rows<MM, CAP, WPB><<<(n + (WPB) - 1) / (WPB), (WPB) * 64, 0, s>>>(n, A.rp, A.ci, A.v, tpos, steps, \
                                                                               step, eps, mcap, cnt, pci, pv, flags)
    if (mcap <= 16 && bound <= 256) AFSAI_LAUNCH(16, 256, 4);
    else if (bound <= 256) AFSAI_LAUNCH(kAfsaiMaxM, 256, 4);
    else if (bound <= 1024) AFSAI_LAUNCH(kAfsaiMaxM, 1024, 2);
    else AFSAI_LAUNCH(kAfsaiMaxM, kAfsaiMaxCand, 1);
#undef AFSAI_LAUNCH
    HIPC(hipGetLastError());
}

void afsai_compact(const Csr &G, int mcap, const int32_t *pci, const double *pv, hipStream_t s) {
    k_afsai_compact<<<nblocks(G.nr), kBlock, 0, s>>>(G.nr, mcap, pci, pv, G.rp, G.ci, G.v);
    HIPC(hipGetLastError());
}

int xi_bounds(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int variant, int32_t *bnd, int *bmax_wave,
              Pool &tmp, hipStream_t s) {
    int32_t *cs = tmp.alloc<int32_t>(n);
    unsigned long long *d = tmp.alloc<unsigned long long>(2);
    HIPC(hipMemsetAsync(d, 0, 2 * sizeof(unsigned long long), s));
    k_xi_cs<<<nblocks(n), kBlock, 0, s>>>(n, A.rp, A.ci, strong, cf, cs);
    k_xi_bound<<<nblocks(n), kBlock, 0, s>>>(n, A.rp, A.ci, strong, cf, cs, variant, bnd, d);
    HIPC(hipGetLastError());
    unsigned long long h[2] = {0, 0};
    HIPC(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    auto clamp = [](unsigned long long x) { return x > (unsigned long long)INT32_MAX ? INT32_MAX : (int)x; };
    *bmax_wave = clamp(h[1]);
    return clamp(h[0]);
}

template <bool FILL>
static void xi_launch(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int variant, const int32_t *bnd,
                      int bmax, const int64_t *cmap, int32_t *cnt, const int32_t *prp, int32_t *pci, double *pv,
                      int32_t *flags, hipStream_t s) {
    // bmax: largest bound of the rows the row-group kernels take (-1: none
    // but those of the thread kernel)
    k_xi_simple<FILL><<<nblocks(n), kBlock, 0, s>>>(n, cf, bnd, cmap, cnt, prp, pci, pv);
    k_xi_thread<kXiCapThread, FILL><<<nblocks(n), kBlock, 0, s>>>(n, A.rp, A.ci, A.v, strong, cf, bnd, variant,
                                                                      cmap, cnt, prp, pci, pv, flags);
    if (bmax >= 1)
        k_xi_rows<kXiCapSmall, 3 * kXiCapSmall / 2, 4, 64, FILL><<<(n + 3) / 4, 256, 0, s>>>(
            n, A.rp, A.ci, A.v, strong, cf, bnd, 1, kXiCapSmall, variant, cmap, cnt, prp, pci, pv, flags);
    if (bmax > kXiCapSmall)
        k_xi_rows<kXiCapMid, 3 * kXiCapMid / 2, 1, 256, FILL><<<n, 256, 0, s>>>(
            n, A.rp, A.ci, A.v, strong, cf, bnd, kXiCapSmall + 1, kXiCapMid, variant, cmap, cnt, prp, pci, pv,
            flags);
    if (bmax > kXiCapMid)
        k_xi_rows<kXiCapGroup, 3 * kXiCapGroup / 2, 1, 256, FILL><<<n, 256, 0, s>>>(
            n, A.rp, A.ci, A.v, strong, cf, bnd, kXiCapMid + 1, kXiCapGroup, variant, cmap, cnt, prp, pci, pv,
            flags);
    HIPC(hipGetLastError());
}

void xi_count(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int variant, const int32_t *bnd, int bmax,
              int32_t *cnt, int32_t *flags, hipStream_t s) {
    // bmax: largest bound over the rows the row-group kernels take
    if (bmax > kXiCapGroup) fail(CAMG_E_ARG, "interpolation: a row has more than 2048 candidate coarse points");
    xi_launch<false>(n, A, strong, cf, variant, bnd, bmax, nullptr, cnt, nullptr, nullptr, nullptr, flags, s);
}

void xi_fill(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int variant, const int32_t *bnd, int bmax,
             const int64_t *cmap, const int32_t *prp, int32_t *pci, double *pv, int32_t *flags, hipStream_t s) {
    xi_launch<true>(n, A, strong, cf, variant, bnd, bmax, cmap, nullptr, prp, pci, pv, flags, s);
}

void bamg_orthonormalize(int n, int nt, double *V, Pool &tmp, hipStream_t s) {
    if (nt < 1 || nt > kBamgNt) fail(CAMG_E_ARG, "test space: 1 to 8 vectors");
    double *G = tmp.alloc<double>((size_t)nt * nt);
    k_gram_tiled<<<1, kGramThreads, 0, s>>>(n, nt, nt, 1, V, nt, V, nullptr, nt, G, nullptr, nt);
    HIPC(hipGetLastError());
    double g[kBamgNt * kBamgNt];
    HIPC(hipMemcpyAsync(g, G, sizeof(double) * nt * nt, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    // G = L L^T, column by column (the CPU reference's operations)
    double gmax = 0.0;
    for (int a = 0; a < nt; ++a) gmax = g[a * nt + a] > gmax ? g[a * nt + a] : gmax;
    for (int j = 0; j < nt; ++j) {
        double d = g[j * nt + j];
        for (int k = 0; k < j; ++k) d = d - g[j * nt + k] * g[j * nt + k];
        if (!(d > 1e-12 * gmax)) fail(CAMG_E_ARG, "test space vectors are linearly dependent");
        const double ljj = std::sqrt(d);
        g[j * nt + j] = ljj;
        for (int i = j + 1; i < nt; ++i) {
            double t = g[i * nt + j];
            for (int k = 0; k < j; ++k) t = t - g[i * nt + k] * g[j * nt + k];
            g[i * nt + j] = t / ljj;
        }
    }
    BamgL L;
    for (int k = 0; k < nt * nt; ++k) L.l[k] = g[k];
    k_ortho_rows<<<nblocks(n), kBlock, 0, s>>>(n, nt, L, V);
    HIPC(hipGetLastError());
}

void bamg_rows(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int nt, const double *V, int lmin,
               int lmax, double eps, double mu, const int64_t *cmap, int32_t *cnt, int32_t *tci, double *tv,
               int32_t *flags, hipStream_t s) {
    k_bamg_rows<<<n, kWave, 0, s>>>(n, A.rp, A.ci, strong, cf, nt, V, lmin, lmax, eps, mu, cmap, cnt, tci, tv,
                                     flags);
    HIPC(hipGetLastError());
}

void bamg_compact(int n, int nt, const int32_t *tci, const double *tv, const Csr &P, hipStream_t s) {
    k_bamg_compact<<<nblocks(n), kBlock, 0, s>>>(n, nt, tci, tv, P.rp, P.ci, P.v);
    HIPC(hipGetLastError());
}

void bamg_gather_tv(int n, int nt, const int8_t *cf, const int64_t *cmap, const double *V, double *Vc, hipStream_t s) {
    k_gather_tv<<<nblocks(n), kBlock, 0, s>>>(n, nt, cf, cmap, V, Vc);
    HIPC(hipGetLastError());
}

void psmooth(const Csr &A, const double *dinv, double omega, Csr &P, Pool &out, Pool &tmp, hipStream_t s) {
    Csr AP;
    spgemm(A, P, AP, tmp, tmp, s);
    const int n = P.nr;
    int32_t *cnt = tmp.alloc<int32_t>(n);
    k_psmooth<false><<<nblocks(n), kBlock, 0, s>>>(n, P.rp, P.ci, P.v, AP.rp, AP.ci, AP.v, dinv, omega, cnt, nullptr,
                                                   nullptr, nullptr);
    HIPC(hipGetLastError());
    int64_t *rp64 = tmp.alloc<int64_t>((size_t)n + 1);
    scan_i32_to_i64(cnt, rp64, n, tmp, s);
    int64_t nnz = 0;
    HIPC(hipMemcpyAsync(&nnz, rp64 + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (nnz > INT32_MAX) fail(CAMG_E_NOMEM, "smoothed prolongation has 2^31 or more entries");
    Csr Ps;
    Ps.nr = n;
    Ps.nc = P.nc;
    Ps.nnz = nnz;
    Ps.rp = out.alloc<int32_t>((size_t)n + 1);
    narrow_i64(rp64, Ps.rp, n, s);
    Ps.ci = out.alloc<int32_t>(padded(nnz));
    Ps.v = out.alloc<double>(padded(nnz));
    k_psmooth<true><<<nblocks(n), kBlock, 0, s>>>(n, P.rp, P.ci, P.v, AP.rp, AP.ci, AP.v, dinv, omega, nullptr, Ps.rp,
                                                  Ps.ci, Ps.v);
    HIPC(hipGetLastError());
    P = Ps;
}

void pfilter(Csr &P, double rho, int nt, const double *W, Pool &out, Pool &tmp, hipStream_t s) {
    const int n = P.nr;
    if (nt < 1 || nt > kBamgNt) fail(CAMG_E_ARG, "filter: 1 to 8 test vectors");
    int32_t *cnt = tmp.alloc<int32_t>(n), *flags = tmp.alloc<int32_t>(3);
    int32_t *tci = tmp.alloc<int32_t>(padded(P.nnz));
    double *tvv = tmp.alloc<double>(padded(P.nnz));
    HIPC(hipMemsetAsync(flags, 0, 3 * sizeof(int32_t), s));
    k_pfilter<<<n, kWave, 0, s>>>(n, P.rp, P.ci, P.v, rho, nt, W, cnt, tci, tvv, flags);
    HIPC(hipGetLastError());
    int32_t hf[3];
    HIPC(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hf[2]) fail(CAMG_E_ARG, "filter: a row of P has more than 1024 entries");
    int64_t *rp64 = tmp.alloc<int64_t>((size_t)n + 1);
    scan_i32_to_i64(cnt, rp64, n, tmp, s);
    Csr F;
    F.nr = n;
    F.nc = P.nc;
    int64_t fnnz = 0;
    HIPC(hipMemcpyAsync(&fnnz, rp64 + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    F.nnz = fnnz;
    F.rp = out.alloc<int32_t>((size_t)n + 1);
    narrow_i64(rp64, F.rp, n, s);
    F.ci = out.alloc<int32_t>(padded(F.nnz));
    F.v = out.alloc<double>(padded(F.nnz));
    k_compact_rows<<<nblocks(n), kBlock, 0, s>>>(n, P.rp, tci, tvv, F.rp, F.ci, F.v);
    HIPC(hipGetLastError());
    P = F;
}

void fill_ones(int n, double *x, hipStream_t s) {
    k_fill_ones<<<nblocks(n), kBlock, 0, s>>>(n, x);
    HIPC(hipGetLastError());
}

double fsai_rayleigh(const Csr &A, const Csr &G, const Csr &Gt, uint64_t seed, int level, Pool &tmp,
                     hipStream_t s) {
    const int n = A.nr;
    double *v = tmp.alloc<double>(n), *t = tmp.alloc<double>(n), *u = tmp.alloc<double>(n), *w = tmp.alloc<double>(n);
    const int nb = std::max(1, std::min(kPwGrid, (n + kBlock - 1) / kBlock));
    double *part = tmp.alloc<double>(3 * (size_t)nb), *st = tmp.alloc<double>(2);
    const unsigned g = (unsigned)nblocks(n);
    k_pw_start<<<g, kBlock, 0, s>>>(n, seed, level, v);
    auto spmv = [&](const Csr &M, const double *x, double *y) {
        const int gl = std::min(group_lanes(n, M.nnz), kOrderedLanes);
        CAMG_G_SWITCH(gl, (k_pw_spmv<G><<<group_blocks(n, G), kBlock, 0, s>>>(n, M.rp, M.ci, M.v, x, y)));
    };
    for (int k = 0; k < kFsaiPowerSteps; ++k) {
        spmv(Gt, v, t);
        spmv(A, t, u);
        spmv(G, u, w);
        k_pw_dots<<<nb, kBlock, 0, s>>>(n, v, w, part);
        k_pw_fin<<<1, kBlock, 0, s>>>(nb, part, st);
        k_pw_scale<<<g, kBlock, 0, s>>>(n, w, st, v);
    }
    HIPC(hipGetLastError());
    double rq = 0.0;
    HIPC(hipMemcpyAsync(&rq, st, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    return rq;
}

int max_row_length(int n, const int32_t *rp, Pool &tmp, hipStream_t s) {
    int32_t *d = tmp.alloc<int32_t>(1);
    HIPC(hipMemsetAsync(d, 0, sizeof(int32_t), s));
    k_max_row<<<nblocks(n), kBlock, 0, s>>>(n, rp, d);
    HIPC(hipGetLastError());
    int32_t h = 0;
    HIPC(hipMemcpyAsync(&h, d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    return h;
}


void srqm(const Csr &A, const double *dinv, const Csr *G, const Csr *Gt, int nt, double *V, int iters, Pool &tmp,
          hipStream_t s) {
    const int n = A.nr, m = 2 * nt;
    if (nt < 1 || nt > kBamgNt) fail(CAMG_E_ARG, "SRQM: 1 to 8 test vectors");
    double *S = tmp.alloc<double>((size_t)n * m), *AS = tmp.alloc<double>((size_t)n * m);
    double *R = G ? tmp.alloc<double>((size_t)n * nt) : nullptr;
    double *Y = G ? tmp.alloc<double>((size_t)n * nt) : nullptr;
    double *T = tmp.alloc<double>(kBamgNt * kBamgNt);
    double *Gs = tmp.alloc<double>(kSrqmM * kSrqmM), *Hs = tmp.alloc<double>(kSrqmM * kSrqmM);
    double *Z = tmp.alloc<double>(kSrqmM * kBamgNt);
    int32_t *K = tmp.alloc<int32_t>(kSrqmM + 1);  // kept columns, then their count
    const unsigned nb = (unsigned)(((size_t)n * nt + kBlock - 1) / kBlock);  // blocks for n x nt threads
    k_copy_block<<<nb, kBlock, 0, s>>>(n, nt, V, nt, S, m);
    for (int it = 0; it < iters; ++it) {
        k_csr_block<<<nb, kBlock, 0, s>>>(n, A.rp, A.ci, A.v, nt, S, m, AS, m);
        k_gram_tiled<<<1, kGramThreads, 0, s>>>(n, nt, nt, 0, S, m, AS, nullptr, m, T, nullptr, nt);
        if (G) {
            k_srqm_resid<<<nblocks(n), kBlock, 0, s>>>(n, nt, m, S, AS, T, nullptr, R, nt);
            k_csr_block<<<nb, kBlock, 0, s>>>(n, G->rp, G->ci, G->v, nt, R, nt, Y, nt);
            k_csr_block<<<nb, kBlock, 0, s>>>(n, Gt->rp, Gt->ci, Gt->v, nt, Y, nt, S + nt, m);
        } else {
            k_srqm_resid<<<nblocks(n), kBlock, 0, s>>>(n, nt, m, S, AS, T, dinv, S + nt, m);
        }
        k_csr_block<<<nb, kBlock, 0, s>>>(n, A.rp, A.ci, A.v, nt, S + nt, m, AS + nt, m);
        k_gram_tiled<<<2, kGramThreads, 0, s>>>(n, m, m, 1, S, m, S, AS, m, Gs, Hs, m);
        k_srqm_rr<<<1, kWave, 0, s>>>(nt, Gs, Hs, K, Z, K + kSrqmM);
        HIPC(hipGetLastError());
        int32_t mk = 0;
        HIPC(hipMemcpyAsync(&mk, K + kSrqmM, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if (mk <= nt) break;  // W adds no direction: V stays
        k_srqm_combine<<<nblocks(n), kBlock, 0, s>>>(n, nt, m, K, K + kSrqmM, Z, S);
    }
    k_copy_block<<<nb, kBlock, 0, s>>>(n, nt, S, m, V, nt);
    HIPC(hipGetLastError());
}
}  // namespace camg
