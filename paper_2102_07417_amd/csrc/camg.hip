// C-ABI of libcamg: hierarchy set-up (Alg. "AMG Set-up"), V-cycle
// (Alg. "AMG application in a V-cycle") and PCG drivers.  Host code only
// orchestrates; every step of set-up and solve runs in the kernels of
// setup.hip, spgemm.hip and solve.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace camg {

static thread_local std::string g_last_error;

void fail(camg_status s, const std::string &msg) { throw Error{s, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        fail(CAMG_E_NOMEM, std::string(what) + ": " + hipGetErrorString(e));
    fail(CAMG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {
constexpr size_t kChunk = (size_t)16 << 20;     // packing chunk
constexpr size_t kOwnBlock = (size_t)4 << 20;   // requests of this size or more get their own block
constexpr size_t kCacheCap = (size_t)4 << 30;   // scratch cache per device
std::mutex g_cache_mu;
std::multimap<size_t, Pool::Block> g_cache;     // free scratch blocks by size
size_t g_cache_bytes[64] = {};

void drain_cache(int dev) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
        if (it->second.device == dev) {
            (void)hipFree(it->second.p);
            g_cache_bytes[dev & 63] -= it->second.size;
            it = g_cache.erase(it);
        } else {
            ++it;
        }
    }
}
}  // namespace

Pool::Block Pool::get(size_t size) {
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        // smallest cached block that fits, if it is not much larger
        for (auto it = g_cache.lower_bound(size); it != g_cache.end() && it->first <= 2 * size + kChunk; ++it)
            if (it->second.device == dev) {
                Block bl = it->second;
                g_cache_bytes[dev & 63] -= bl.size;
                g_cache.erase(it);
                return bl;
            }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, size);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        drain_cache(dev);
        e = hipMalloc(&p, size);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(CAMG_E_NOMEM, "device allocation of " + std::to_string(size) + " bytes failed");
    }
    return Block{p, size, dev};
}

void *Pool::raw(size_t nbytes) {
    if (nbytes == 0) nbytes = 1;
    nbytes = (nbytes + 255) & ~(size_t)255;
    bytes += (int64_t)nbytes;
    if (nbytes <= left_) {
        void *p = cur_;
        cur_ += nbytes;
        left_ -= nbytes;
        return p;
    }
    if (nbytes >= kOwnBlock) {
        blocks_.push_back(get(nbytes));
        return blocks_.back().p;
    }
    blocks_.push_back(get(kChunk));
    cur_ = static_cast<char *>(blocks_.back().p) + nbytes;
    left_ = blocks_.back().size - nbytes;
    return blocks_.back().p;
}

void Pool::release() {
    if (blocks_.empty()) return;
    bool keep = true;
    if (scratch_) {
        if (hipStreamSynchronize(stream_) != hipSuccess) keep = false;  // the stream's work on these blocks is done
    } else {
        // a handle's or an engine's blocks, which any stream may still use:
        // wait for the devices they live on, as hipFree would
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) keep = false;
        std::vector<int> devs;
        for (const Block &bl : blocks_)
            if (std::find(devs.begin(), devs.end(), bl.device) == devs.end()) devs.push_back(bl.device);
        for (int d : devs)
            if (hipSetDevice(d) != hipSuccess || hipDeviceSynchronize() != hipSuccess) keep = false;
        if (cur >= 0) (void)hipSetDevice(cur);
    }
    if (!keep) (void)hipGetLastError();
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (const Block &bl : blocks_) {
            if (keep && g_cache_bytes[bl.device & 63] + bl.size <= kCacheCap) {
                g_cache.emplace(bl.size, bl);
                g_cache_bytes[bl.device & 63] += bl.size;
            } else {
                (void)hipFree(bl.p);
            }
        }
    }
    blocks_.clear();
    cur_ = nullptr;
    left_ = 0;
    bytes = 0;
}

namespace {

struct BusyGuard {
    Hier *h;
    explicit BusyGuard(Hier *hh) : h(hh) {
        int expect = 0;
        if (!h->busy.compare_exchange_strong(expect, 1)) fail(CAMG_E_BUSY, "handle is in use by another call");
    }
    ~BusyGuard() { h->busy.store(0); }
};

template <class F>
camg_status guarded(F &&f) {
    try {
        f();
        return CAMG_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return CAMG_E_NOMEM;
    } catch (...) {
        g_last_error = "unexpected exception";
        return CAMG_E_DEVICE;
    }
}

template <class T>
T read1(const T *d, hipStream_t s) {
    T v;
    HIPC(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    return v;
}

void check_params(const camg_params &p) {
    if (!(p.theta >= 0.0 && p.theta <= 1.0)) fail(CAMG_E_ARG, "theta must lie in [0, 1]");
    if (p.nu_pre < 1 || p.nu_pre > 8 || p.nu_post < 1 || p.nu_post > 8)
        fail(CAMG_E_ARG, "nu_pre and nu_post must lie in [1, 8]");
    if (p.max_levels < 1 || p.max_levels > CAMG_MAX_LEVELS) fail(CAMG_E_ARG, "max_levels must lie in [1, 32]");
    if (p.max_coarse < 1) fail(CAMG_E_ARG, "max_coarse must be >= 1");
    if (p.max_iter < 0) fail(CAMG_E_ARG, "max_iter must be >= 0");
    if (p.precision != CAMG_FP64 && p.precision != CAMG_MIXED_FP32) fail(CAMG_E_ARG, "unknown precision");
    if (!std::isfinite(p.omega)) fail(CAMG_E_ARG, "omega must be finite");
    if (p.smoother != CAMG_SMOOTH_JACOBI && p.smoother != CAMG_SMOOTH_FSAI && p.smoother != CAMG_SMOOTH_FSAI_JACOBI &&
        p.smoother != CAMG_SMOOTH_AFSAI)
        fail(CAMG_E_ARG, "unknown smoother");
    if (p.smoother == CAMG_SMOOTH_AFSAI &&
        (p.afsai_steps < 0 || p.afsai_step < 1 || (int64_t)p.afsai_steps * p.afsai_step + 1 > CAMG_AFSAI_MAXM ||
         !(p.afsai_eps >= 0.0)))
        fail(CAMG_E_ARG, "aFSAI: need afsai_steps >= 0, afsai_step >= 1, afsai_steps * afsai_step + 1 <= 32 and "
                         "afsai_eps >= 0");
    if (p.interp < CAMG_INTERP_DIRECT || p.interp > CAMG_INTERP_BAMG) fail(CAMG_E_ARG, "unknown interpolation");
    if (p.interp == CAMG_INTERP_BAMG &&
        (p.bamg_lmin < 1 || p.bamg_lmax < p.bamg_lmin || p.bamg_lmax > 2 || std::isnan(p.bamg_eps) || std::isnan(p.bamg_mu)))
        fail(CAMG_E_ARG, "BAMG: need 1 <= bamg_lmin <= bamg_lmax <= 2 and eps, mu not NaN");
    if (p.rap_chunk < 0) fail(CAMG_E_ARG, "rap_chunk must be >= 0");
    if (p.psmooth != 0 && p.psmooth != 1) fail(CAMG_E_ARG, "psmooth must be 0 or 1");
    if (!(p.pfilter > 0.0)) fail(CAMG_E_ARG, "pfilter must be > 0");
    if (p.srqm_iters < 0 || p.srqm_iters > 100) fail(CAMG_E_ARG, "srqm_iters must lie in [0, 100]");
    if (p.srqm_iters > 0 && p.interp != CAMG_INTERP_BAMG)
        fail(CAMG_E_ARG, "srqm_iters refines the BAMG test space: it needs CAMG_INTERP_BAMG");
}

// ---------------------------------------------------------------- set-up
void validate_input(Hier &h, int n, int64_t nnz, const Csr &A, int32_t *tpos, Pool &tmp, hipStream_t s) {
    int32_t *flags = tmp.alloc<int32_t>(8);
    unsigned long long *amax = tmp.alloc<unsigned long long>(1);
    HIPC(hipMemsetAsync(flags, 0, 8 * sizeof(int32_t), s));
    HIPC(hipMemsetAsync(amax, 0, sizeof(unsigned long long), s));
    validate_rowptr(n, nnz, A.rp, flags, s);
    int32_t hf[8];
    HIPC(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hf[0]) fail(CAMG_E_CSR, "row pointer is not 0-based and non-decreasing up to nnz");
    validate_rows(n, nnz, A.rp, A.ci, A.v, flags, amax, s);
    HIPC(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hf[1]) fail(CAMG_E_CSR, "column index out of range or not strictly increasing within a row");
    if (hf[2]) fail(CAMG_E_CSR, "non-finite matrix value");
    if (hf[3]) fail(CAMG_E_CSR, "a diagonal entry is missing");
    validate_sym(n, nnz, A.rp, A.ci, A.v, amax, flags, tpos, s);
    HIPC(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hf[4]) fail(CAMG_E_CSR, "matrix is not symmetric (pattern or values beyond 1e-12 max|a|)");
    if (hf[5]) fail(CAMG_E_NOT_SPD, "non-positive diagonal entry");
    (void)h;
}

void alloc_f32_copy(Pool &pool, Csr &M, hipStream_t s) {
    M.v32 = pool.alloc<float>(padded(M.nnz));
    to_f32(M.nnz, M.v, M.v32, s);
}

// Launch shapes of several matrices with two synchronisations in all (the
// longest rows, then the tile-base modes) instead of two per matrix.
void make_cfgs(Hier &h, const std::vector<std::pair<const Csr *, RowCfg *>> &ms, Pool &tmp, hipStream_t s) {
    const int nm = (int)ms.size();
    if (nm == 0) return;
    int32_t *d = tmp.alloc<int32_t>(3 * (size_t)nm);  // longest row, then two flags per matrix
    HIPC(hipMemsetAsync(d, 0, 3 * sizeof(int32_t) * (size_t)nm, s));
    for (int k = 0; k < nm; ++k) max_row_length_async(ms[k].first->nr, ms[k].first->rp, d + k, s);
    std::vector<int32_t> hd(3 * (size_t)nm);
    HIPC(hipMemcpyAsync(hd.data(), d, sizeof(int32_t) * (size_t)nm, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    std::vector<int32_t *> tbs(nm, nullptr);
    for (int k = 0; k < nm; ++k) {
        const Csr &M = *ms[k].first;
        RowCfg &c = *ms[k].second;
        c = choose_cfg(M.nr, M.nnz, hd[k]);
        if (!c.tile) continue;
        c.tstart = h.pool.alloc<int32_t>((size_t)c.ntiles + 1);
        tile_starts(M.nr, M.rp, c.W, c.ntiles, c.tstart, s);
        tbs[k] = h.pool.alloc<int32_t>((size_t)c.ntiles * kTileWins);
        tile_bases_async(c.ntiles, c.tstart, M.rp, M.ci, tbs[k], d + nm + 2 * k, s);
    }
    HIPC(hipMemcpyAsync(hd.data() + nm, d + nm, 2 * sizeof(int32_t) * (size_t)nm, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int k = 0; k < nm; ++k) {
        RowCfg &c = *ms[k].second;
        if (!c.tile || c.ntiles <= 0) continue;
        const int32_t *f = hd.data() + nm + 2 * k;
        const int mode = f[1] == 0 ? 1 : f[0] == 0 ? 2 : 0;
        if (!mode) continue;
        // 16-bit column words (window, offset) per tile: 10 bytes per FP64
        // nonzero instead of 12 (6 instead of 8 in FP32) where the tiles
        // allow them
        const Csr &M = *ms[k].first;
        c.tbase = tbs[k];
        c.off = h.pool.alloc<uint16_t>(padded(M.nnz));
        c.off_mode = mode;
        tile_diffs(c.ntiles, c.tstart, M.rp, M.ci, c.tbase, c.off, mode, s);
        c.use_off = h.compact_cols;
    }
}

void build_hierarchy(Hier &h, int n, const int32_t *rp, const int32_t *ci, const double *v, int nt,
                     const double *V, bool host_in, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const camg_params &prm = h.prm;
    Pool tmp(s);
    // wall time per phase, taken at the stream synchronisations that end
    // them; with CAMG_LOG_SETUP set in the environment each phase is also
    // printed to stderr as it ends
    static const char *const kPhase[8] = {"input", "smoother", "strength+pmis", "interpolation",
                                          "transpose", "galerkin", "last level", "solve buffers"};
    static const bool log_setup = std::getenv("CAMG_LOG_SETUP") != nullptr;
    auto tp = t0;
    int cur_level = 0;
    auto phase = [&](int k) {
        HIPC(hipStreamSynchronize(s));
        const auto t = std::chrono::steady_clock::now();
        const double dt = std::chrono::duration<double, std::milli>(t - tp).count();
        h.phase_ms[k] += dt;
        tp = t;
        if (log_setup) {
            std::fprintf(stderr, "[camg setup] level %d %s %.1f ms\n", cur_level, kPhase[k], dt);
            std::fflush(stderr);
        }
    };
    int64_t nnz;
    if (host_in) nnz = rp[n];
    else nnz = read1(rp + n, s);
    if (nnz < 0) fail(CAMG_E_CSR, "row_ptr[n] is negative");

    h.lev.clear();
    h.lev.emplace_back();
    {
        Csr &A = h.lev[0].A;
        A.nr = A.nc = n;
        A.nnz = nnz;
        A.rp = h.pool.alloc<int32_t>((size_t)n + 1);
        A.ci = h.pool.alloc<int32_t>(padded(nnz));
        A.v = h.pool.alloc<double>(padded(nnz));
        const hipMemcpyKind k = host_in ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        HIPC(hipMemcpyAsync(A.rp, rp, sizeof(int32_t) * ((size_t)n + 1), k, s));
        HIPC(hipMemcpyAsync(A.ci, ci, sizeof(int32_t) * (size_t)nnz, k, s));
        HIPC(hipMemcpyAsync(A.v, v, sizeof(double) * (size_t)nnz, k, s));
    }
    int32_t *tpos = tmp.alloc<int32_t>(std::max<int64_t>(nnz, 1));
    validate_input(h, n, nnz, h.lev[0].A, tpos, tmp, s);
    // BAMG: the level's test space (orthonormal basis of V on level 0)
    double *tv = nullptr;
    if (prm.interp == CAMG_INTERP_BAMG) {
        tv = tmp.alloc<double>((size_t)n * nt);
        HIPC(hipMemcpyAsync(tv, V, sizeof(double) * (size_t)n * nt,
                            host_in ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
        bamg_orthonormalize(n, nt, tv, tmp, s);
    }
    phase(0);

    int32_t *flags = tmp.alloc<int32_t>(8);
    unsigned long long *qmax = tmp.alloc<unsigned long long>(1);
    int32_t *und = tmp.alloc<int32_t>(2);  // undecided-point flags of two PMIS rounds
    for (int l = 0;; ++l) {
        cur_level = l;
        const int nl = h.lev[l].A.nr;
        if (nl <= prm.max_coarse || l == prm.max_levels - 1) break;
        Level &L = h.lev[l];
        const int64_t nz = L.A.nnz;
        Pool lt(s);  // per-level temporaries
        if (l > 0) {
            tpos = lt.alloc<int32_t>(std::max<int64_t>(nz, 1));
            transpose_positions(nl, nz, L.A.rp, L.A.ci, tpos, s);
        }
        // Jacobi weights (eq. smoother)
        L.dinv = h.pool.alloc<double>(nl);
        L.wd = h.pool.alloc<double>(nl);
        HIPC(hipMemsetAsync(flags, 0, 8 * sizeof(int32_t), s));
        diag_gershgorin(nl, nz, L.A.rp, L.A.ci, L.A.v, L.dinv, qmax, flags, s);
        int32_t hf[8];
        unsigned long long hq;
        HIPC(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(&hq, qmax, sizeof(hq), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if (hf[5]) fail(CAMG_E_NOT_SPD, "non-positive diagonal on level " + std::to_string(l));
        double rho;
        std::memcpy(&rho, &hq, sizeof(rho));
        L.omega = prm.omega > 0.0 ? prm.omega : (4.0 / 3.0) / rho;
        const double w_jacobi = L.omega;  // also the weight of prolongation smoothing
        scale_vec(nl, L.omega, L.dinv, L.wd, s);
        L.awd = h.pool.alloc<double>(padded(nz));
        scale_columns(L.A, L.wd, L.awd, s);
        // FSAI on this level: always with CAMG_SMOOTH_FSAI; with
        // CAMG_SMOOTH_FSAI_JACOBI when no row has more than kFsaiMaxRow
        // entries on or below the diagonal (Jacobi otherwise)
        int32_t *gcnt = nullptr;
        int mmax = 0;
        if (prm.smoother == CAMG_SMOOTH_FSAI || prm.smoother == CAMG_SMOOTH_FSAI_JACOBI) {
            gcnt = lt.alloc<int32_t>(nl);
            mmax = fsai_counts(nl, L.A.rp, L.A.ci, gcnt, lt, s);
        }
        L.fsai = prm.smoother == CAMG_SMOOTH_FSAI || (prm.smoother == CAMG_SMOOTH_FSAI_JACOBI && mmax <= kFsaiMaxRow);
        // adaptive FSAI: rows padded to mcap slots; Jacobi on a level where a
        // candidate set outgrows the kernel's 2048 entries
        const bool adaptive = prm.smoother == CAMG_SMOOTH_AFSAI;
        const int mcap = adaptive ? prm.afsai_steps * prm.afsai_step + 1 : 0;
        int32_t *apci = nullptr;
        double *apv = nullptr;
        if (adaptive) {
            gcnt = lt.alloc<int32_t>(nl);
            apci = lt.alloc<int32_t>((size_t)nl * mcap);
            apv = lt.alloc<double>((size_t)nl * mcap);
            const int maxrow = max_row_length(nl, L.A.rp, lt, s);
            HIPC(hipMemsetAsync(flags, 0, 8 * sizeof(int32_t), s));
            afsai_rows(L.A, tpos, maxrow, prm.afsai_steps, prm.afsai_step, prm.afsai_eps, gcnt, apci, apv, flags, s);
            int32_t af[8];
            HIPC(hipMemcpyAsync(af, flags, sizeof(af), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            if (af[4]) fail(CAMG_E_DEVICE, "aFSAI: candidate capacity of the launched tier exceeded");
            if (af[7]) fail(CAMG_E_NOT_SPD, "aFSAI: a local matrix is not positive definite on level " +
                                                std::to_string(l));
            L.fsai = af[6] == 0;
        }
        if (L.fsai) {
            // FSAI factor (static on the lower pattern of A_l, or the
            // adaptive one), its transpose, omega (eq. smo, eq. smoother)
            int64_t *grp64 = lt.alloc<int64_t>((size_t)nl + 1);
            scan_i32_to_i64(gcnt, grp64, nl, lt, s);
            Csr &G = L.G;
            G.nr = G.nc = nl;
            G.nnz = read1(grp64 + nl, s);
            G.rp = h.pool.alloc<int32_t>((size_t)nl + 1);
            narrow_i64(grp64, G.rp, nl, s);
            G.ci = h.pool.alloc<int32_t>(padded(G.nnz));
            G.v = h.pool.alloc<double>(padded(G.nnz));
            if (adaptive) {
                afsai_compact(G, mcap, apci, apv, s);
            } else {
                HIPC(hipMemsetAsync(flags, 0, 8 * sizeof(int32_t), s));
                fsai_rows(L.A, G, mmax, flags, s);
                int32_t gf[8];
                HIPC(hipMemcpyAsync(gf, flags, sizeof(gf), hipMemcpyDeviceToHost, s));
                HIPC(hipStreamSynchronize(s));
                if (gf[6]) fail(CAMG_E_ARG, "FSAI: a row has more than 192 entries on or below the diagonal");
                if (gf[7]) fail(CAMG_E_NOT_SPD, "FSAI: a local matrix is not positive definite on level " +
                                                    std::to_string(l));
            }
            Csr &Gt = L.Gt;
            Gt.nr = Gt.nc = nl;
            Gt.nnz = G.nnz;
            int32_t *gcc = lt.alloc<int32_t>(nl);
            column_counts(G, gcc, s);
            int64_t *gtrp64 = lt.alloc<int64_t>((size_t)nl + 1);
            scan_i32_to_i64(gcc, gtrp64, nl, lt, s);
            Gt.rp = h.pool.alloc<int32_t>((size_t)nl + 1);
            narrow_i64(gtrp64, Gt.rp, nl, s);
            Gt.ci = h.pool.alloc<int32_t>(padded(Gt.nnz));
            Gt.v = h.pool.alloc<double>(padded(Gt.nnz));
            transpose_csr(G, Gt, lt, s);
            if (prm.omega > 0.0) {
                L.omega = prm.omega;
            } else {
                L.omega = (4.0 / 3.0) / fsai_rayleigh(L.A, G, Gt, prm.seed, l, lt, s);
            }
        }
        if (prm.interp == CAMG_INTERP_BAMG && l == 0 && prm.srqm_iters > 0) {
            // refine the level-0 test space with the smoother just built
            // (counted in the smoother phase), then make it orthonormal again
            const bool fs = L.fsai;
            srqm(L.A, L.dinv, fs ? &L.G : nullptr, fs ? &L.Gt : nullptr, nt, tv, prm.srqm_iters, lt, s);
            bamg_orthonormalize(nl, nt, tv, lt, s);
        }
        phase(1);
        // strength and PMIS
        L.strong = h.pool.alloc<uint8_t>(std::max<int64_t>(nz, 1));
        L.stcnt = h.pool.alloc<int32_t>(nl);
        L.cf = h.pool.alloc<int8_t>(nl);
        strength(nl, nz, L.A.rp, L.A.ci, L.A.v, tpos, prm.theta, L.strong, L.stcnt, s);
        uint64_t *u = lt.alloc<uint64_t>(nl);
        int8_t *newc = lt.alloc<int8_t>(nl);
        pmis_init(nl, L.stcnt, prm.seed, l, u, L.cf, und, s);
        int32_t hund = read1(und, s);
        int rounds = 0;
        // two rounds per read-back of the flags (a round after the last one
        // finds no undecided point and changes nothing); rounds counts those
        // that started with undecided points
        while (hund > 0) {
            pmis_round(nl, nz, L.A.rp, L.A.ci, L.strong, tpos, L.stcnt, u, L.cf, newc, und, s);
            pmis_round(nl, nz, L.A.rp, L.A.ci, L.strong, tpos, L.stcnt, u, L.cf, newc, und + 1, s);
            int32_t hu[2];
            HIPC(hipMemcpyAsync(hu, und, sizeof(hu), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            rounds += hu[0] > 0 ? 2 : 1;
            hund = hu[0] > 0 ? hu[1] : 0;
            if (rounds > nl + 1) fail(CAMG_E_DEVICE, "PMIS did not terminate");
        }
        L.rounds = rounds;
        // coarse numbering
        int32_t *isc = lt.alloc<int32_t>(nl);
        int64_t *cmap = lt.alloc<int64_t>((size_t)nl + 1);
        cf_flags(nl, L.cf, isc, s);
        scan_i32_to_i64(isc, cmap, nl, lt, s);
        const int64_t nc = read1(cmap + nl, s);
        if (nc == 0 || nc == nl) break;  // coarsening stalled: this is the last level
        phase(2);
        // interpolation P = [W; I]: direct, the paper's classical,
        // extended+i or hybrid formula, or BAMG over the test space
        Csr &P = L.P;
        P.nr = nl;
        P.nc = (int32_t)nc;
        int32_t *pcnt = lt.alloc<int32_t>(nl);
        int32_t *bnd = nullptr, *xflags = nullptr, *btci = nullptr;
        double *btv = nullptr;
        int bmax = 0;
        if (prm.interp == CAMG_INTERP_DIRECT) {
            interp_count(nl, nz, L.A.rp, L.A.ci, L.strong, L.cf, pcnt, s);
        } else if (prm.interp == CAMG_INTERP_BAMG) {
            btci = lt.alloc<int32_t>((size_t)nl * nt);
            btv = lt.alloc<double>((size_t)nl * nt);
            xflags = lt.alloc<int32_t>(3);
            HIPC(hipMemsetAsync(xflags, 0, 3 * sizeof(int32_t), s));
            bamg_rows(nl, L.A, L.strong, L.cf, nt, tv, prm.bamg_lmin, prm.bamg_lmax, prm.bamg_eps, prm.bamg_mu, cmap,
                      pcnt, btci, btv, xflags, s);
            int32_t hf[3];
            HIPC(hipMemcpyAsync(hf, xflags, sizeof(hf), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            if (hf[2]) fail(CAMG_E_ARG, "BAMG: a row has more than 128 candidate coarse points");
        } else {
            bnd = lt.alloc<int32_t>(nl);
            xflags = lt.alloc<int32_t>(2);
            HIPC(hipMemsetAsync(xflags, 0, 2 * sizeof(int32_t), s));
            xi_bounds(nl, L.A, L.strong, L.cf, prm.interp, bnd, &bmax, lt, s);
            xi_count(nl, L.A, L.strong, L.cf, prm.interp, bnd, bmax, pcnt, xflags, s);
        }
        int64_t *prp64 = lt.alloc<int64_t>((size_t)nl + 1);
        scan_i32_to_i64(pcnt, prp64, nl, lt, s);
        P.nnz = read1(prp64 + nl, s);
        if (P.nnz > INT32_MAX) fail(CAMG_E_ARG, "interpolation has 2^31 or more entries");
        P.rp = h.pool.alloc<int32_t>((size_t)nl + 1);
        narrow_i64(prp64, P.rp, nl, s);
        P.ci = h.pool.alloc<int32_t>(padded(P.nnz));
        P.v = h.pool.alloc<double>(padded(P.nnz));
        if (prm.interp == CAMG_INTERP_DIRECT) {
            interp_fill(nl, nz, L.A.rp, L.A.ci, L.A.v, L.strong, L.cf, cmap, P.rp, P.ci, P.v, s);
        } else if (prm.interp == CAMG_INTERP_BAMG) {
            bamg_compact(nl, nt, btci, btv, P, s);
            // the next level's test space: the rows at the C points
            double *tvc = tmp.alloc<double>((size_t)nc * nt);
            bamg_gather_tv(nl, nt, L.cf, cmap, tv, tvc, s);
            tv = tvc;
        } else {
            xi_fill(nl, L.A, L.strong, L.cf, prm.interp, bnd, bmax, cmap, P.rp, P.ci, P.v, xflags, s);
            int32_t hf[2];
            HIPC(hipMemcpyAsync(hf, xflags, sizeof(hf), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            if (hf[0] || hf[1]) fail(CAMG_E_DEVICE, "interpolation: inconsistent candidate lists");
        }
        // prolongation smoothing and filtering (Section 2, Interpolation and
        // Filtering); the filter keeps P's action on the coarse test space
        // (a unit vector without one)
        if (prm.psmooth) psmooth(L.A, L.dinv, w_jacobi, P, h.pool, lt, s);
        if (prm.pfilter < 1.0) {
            const double *W = tv;
            int ntw = nt;
            if (prm.interp != CAMG_INTERP_BAMG) {
                double *ones = lt.alloc<double>(std::max<int64_t>(nc, 1));
                fill_ones((int)nc, ones, s);
                W = ones;
                ntw = 1;
            }
            pfilter(P, prm.pfilter, ntw, W, h.pool, lt, s);
        }
        phase(3);
        // R = P^T
        Csr &R = L.R;
        R.nr = P.nc;
        R.nc = nl;
        R.nnz = P.nnz;
        int32_t *ccnt = lt.alloc<int32_t>(P.nc);
        column_counts(P, ccnt, s);
        int64_t *rrp64 = lt.alloc<int64_t>((size_t)P.nc + 1);
        scan_i32_to_i64(ccnt, rrp64, P.nc, lt, s);
        R.rp = h.pool.alloc<int32_t>((size_t)P.nc + 1);
        narrow_i64(rrp64, R.rp, P.nc, s);
        R.ci = h.pool.alloc<int32_t>(padded(R.nnz));
        R.v = h.pool.alloc<double>(padded(R.nnz));
        transpose_csr(P, R, lt, s);
        phase(4);
        // Galerkin product A_{l+1} = R (A P)  (eq. AcDef)
        Csr Ac;
        galerkin(L.A, P, R, Ac, prm.rap_chunk, h.pool, lt, s);
        phase(5);
        HIPC(hipStreamSynchronize(s));
        lt.release();
        Level next;
        next.A = Ac;
        h.lev.push_back(next);
    }
    h.nlev = (int)h.lev.size();
    // last level: dense Cholesky and explicit inverse (FP64)
    Level &Lc = h.lev.back();
    h.nL = Lc.A.nr;
    if (h.nL > 8192) fail(CAMG_E_COARSE, "coarsening stalled with " + std::to_string(h.nL) + " unknowns");
    {
        double *D = tmp.alloc<double>((size_t)h.nL * h.nL);
        dense_from_csr(h.nL, Lc.A.rp, Lc.A.ci, Lc.A.v, D, s);
        HIPC(hipMemsetAsync(flags, 0, 8 * sizeof(int32_t), s));
        cholesky_dense(h.nL, D, flags, s);
        int32_t hf[8];
        HIPC(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if (hf[5]) fail(CAMG_E_NOT_SPD, "non-positive pivot in the Cholesky factorisation of the last level");
        h.cinv = h.pool.alloc<double>((size_t)h.nL * h.nL);
        chol_inverse(h.nL, D, h.cinv, s);
    }
    phase(6);
    // launch shapes, work vectors, mixed-precision copies
    const bool mixed = prm.precision == CAMG_MIXED_FP32;
    {
        std::vector<std::pair<const Csr *, RowCfg *>> ms;
        for (int l = 0; l < h.nlev; ++l) {
            Level &L = h.lev[l];
            ms.push_back({&L.A, &L.cA});
            if (l < h.nlev - 1) {
                ms.push_back({&L.P, &L.cP});
                ms.push_back({&L.R, &L.cR});
            }
            if (L.fsai && l < h.nlev - 1) {
                ms.push_back({&L.G, &L.cG});
                ms.push_back({&L.Gt, &L.cGt});
            }
        }
        make_cfgs(h, ms, tmp, s);
    }
    for (int l = 0; l < h.nlev; ++l) {
        Level &L = h.lev[l];
        const int nl = L.A.nr;
        const bool fsai = L.fsai && l < h.nlev - 1;
        if (!mixed) {
            if (l > 0) {
                L.y = h.pool.alloc<double>(nl);
                L.z = h.pool.alloc<double>(nl);
            }
            L.s = h.pool.alloc<double>(nl);
            L.r = h.pool.alloc<double>(nl);
        } else {
            L.y32 = h.pool.alloc<float>(nl);
            L.z32 = h.pool.alloc<float>(nl);
            L.s32 = h.pool.alloc<float>(nl);
            L.r32 = h.pool.alloc<float>(nl);
            if (l < h.nlev - 1) {
                alloc_f32_copy(h.pool, L.A, s);
                alloc_f32_copy(h.pool, L.P, s);
                alloc_f32_copy(h.pool, L.R, s);
                L.wd32 = h.pool.alloc<float>(nl);
                to_f32(nl, L.wd, L.wd32, s);
                L.awd32 = h.pool.alloc<float>(padded(L.A.nnz));
                to_f32(L.A.nnz, L.awd, L.awd32, s);
                if (fsai) {
                    alloc_f32_copy(h.pool, L.G, s);
                    alloc_f32_copy(h.pool, L.Gt, s);
                }
            }
        }
        // extra buffer for more than one smoothing step (FSAI: for u = G d)
        if (prm.nu_pre > 1 || prm.nu_post > 1 || fsai) {
            if (!mixed) L.t = h.pool.alloc<double>(nl);
            else L.t32 = h.pool.alloc<float>(nl);
        }
    }
    const int n0 = h.lev[0].A.nr;
    h.x = h.pool.alloc<double>(n0);
    h.r = h.pool.alloc<double>(n0);
    h.z = h.pool.alloc<double>(n0);
    h.p[0] = h.pool.alloc<double>(n0);
    h.p[1] = h.pool.alloc<double>(n0);
    h.q = h.pool.alloc<double>(n0);
    h.pr2 = h.pool.alloc<double>(kMaxPartials);
    h.prz = h.pool.alloc<double>(kMaxPartials);
    h.ppq = h.pool.alloc<double>(kMaxPartials);
    h.ptmp = h.pool.alloc<double>(kMaxPartials);
    h.st = h.pool.alloc<PcgState>(1);
    h.sc = h.pool.alloc<double>(4);
    HIPC(hipHostMalloc((void **)&h.hflag, 4 * sizeof(int32_t), hipHostMallocMapped));
    HIPC(hipHostGetDevicePointer((void **)&h.hflag_dev, h.hflag, 0));
    HIPC(hipStreamSynchronize(s));
    phase(7);
    h.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- V-cycle
template <class T>
struct VT;
template <>
struct VT<double> {
    static const double *wd(const Level &L) { return L.wd; }
    static const double *awd(const Level &L) { return L.awd; }
    static double *y(Level &L) { return L.y; }
    static double *s(Level &L) { return L.s; }
    static double *r(Level &L) { return L.r; }
    static double *z(Level &L) { return L.z; }
    static double *t(Level &L) { return L.t; }
};
template <>
struct VT<float> {
    static const float *wd(const Level &L) { return L.wd32; }
    static const float *awd(const Level &L) { return L.awd32; }
    static float *y(Level &L) { return L.y32; }
    static float *s(Level &L) { return L.s32; }
    static float *r(Level &L) { return L.r32; }
    static float *z(Level &L) { return L.z32; }
    static float *t(Level &L) { return L.t32; }
};

int32_t *st_count(PcgState *st, size_t off) { return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(st) + off); }

// Pre-smoothing (nu_pre steps from s = 0) and residual on level l.
// Returns the buffer that holds s.
// FSAI pre-smoothing (eq. smo): s = omega G^T G y, then nu_pre - 1 steps
// s += omega G^T G (y - A s) in place, then r = y - A s.  u = G d lives in t,
// d in r.
template <class T, class TY>
T *fsai_pre(Hier &h, Level &L, const TY *y, PcgState *st, hipStream_t s) {
    T *sv = VT<T>::s(L), *tv = VT<T>::t(L), *rv = VT<T>::r(L);
    const T om = (T)L.omega;
    vc_gmul<T, TY>(L.G, L.cG, y, tv, st, s);
    vc_fsai_first<T>(L.Gt, L.cGt, om, tv, sv, st, s);
    for (int it = 1; it < h.prm.nu_pre; ++it) {
        vc_resid<T, TY>(L.A, L.cA, y, sv, rv, st, s);
        vc_gmul<T, T>(L.G, L.cG, rv, tv, st, s);
        vc_fsai_step<T, TY, T, false>(L.Gt, L.cGt, om, tv, sv, nullptr, sv, nullptr, nullptr, st, s);
    }
    vc_resid<T, TY>(L.A, L.cA, y, sv, rv, st, s);
    return sv;
}

// FSAI post-smoothing: nu_post steps, the last one into z (with dot: the
// partials of y.z into h.prz, their count into st->n_rz)
template <class T, class TY, class TZ>
void fsai_post(Hier &h, Level &L, const TY *y, T *sv, TZ *z, bool dot, PcgState *st, hipStream_t s) {
    T *tv = VT<T>::t(L), *rv = VT<T>::r(L);
    const T om = (T)L.omega;
    for (int it = 0; it < h.prm.nu_post; ++it) {
        vc_resid<T, TY>(L.A, L.cA, y, sv, rv, st, s);
        vc_gmul<T, T>(L.G, L.cG, rv, tv, st, s);
        if (it + 1 < h.prm.nu_post)
            vc_fsai_step<T, TY, T, false>(L.Gt, L.cGt, om, tv, sv, nullptr, sv, nullptr, nullptr, st, s);
        else if (dot)
            vc_fsai_step<T, TY, TZ, true>(L.Gt, L.cGt, om, tv, sv, y, z, h.prz,
                                           st_count(st, offsetof(PcgState, n_rz)), st, s);
        else
            vc_fsai_step<T, TY, TZ, false>(L.Gt, L.cGt, om, tv, sv, nullptr, z, nullptr, nullptr, st, s);
    }
}

template <class T, class TY>
T *smooth_pre(Hier &h, Level &L, const TY *y, PcgState *st, hipStream_t s) {
    if (L.fsai) return fsai_pre<T, TY>(h, L, y, st, s);
    T *sv = VT<T>::s(L), *tv = VT<T>::t(L);
    vc_pre<T, TY>(L.A, L.cA, VT<T>::wd(L), VT<T>::awd(L), y, sv, VT<T>::r(L), st, s);
    if (h.prm.nu_pre > 1) {
        for (int it = 1; it < h.prm.nu_pre; ++it) {
            vc_post<T, TY, T, false>(L.A, L.cA, VT<T>::wd(L), y, sv, tv, nullptr, nullptr, st, s);
            std::swap(sv, tv);
        }
        vc_resid<T, TY>(L.A, L.cA, y, sv, VT<T>::r(L), st, s);
    }
    return sv;
}

// Post-smoothing (nu_post steps) into z; with dot the last step also writes
// the partials of y.z into h.prz and their count into st->n_rz.
template <class T, class TY, class TZ>
void smooth_post(Hier &h, Level &L, const TY *y, T *sv, TZ *z, bool dot, PcgState *st, hipStream_t s) {
    if (L.fsai) {
        fsai_post<T, TY, TZ>(h, L, y, sv, z, dot, st, s);
        return;
    }
    T *tv = VT<T>::t(L);
    for (int it = 0; it + 1 < h.prm.nu_post; ++it) {
        T *out = (tv == sv) ? VT<T>::s(L) : tv;
        vc_post<T, TY, T, false>(L.A, L.cA, VT<T>::wd(L), y, sv, out, nullptr, nullptr, st, s);
        sv = out;
    }
    if (dot)
        vc_post<T, TY, TZ, true>(L.A, L.cA, VT<T>::wd(L), y, sv, z, h.prz, st_count(st, offsetof(PcgState, n_rz)),
                                 st, s);
    else
        vc_post<T, TY, TZ, false>(L.A, L.cA, VT<T>::wd(L), y, sv, z, nullptr, nullptr, st, s);
}

// z0 = M y0 with T-valued levels; y0, z0 are FP64 level-0 vectors.  The
// cycle is split in two parts: `head` runs everything up to and including
// the level-0 prolongation, `tail` the level-0 post-smoothing (with dot, the
// partials of y0.z0 land in h.prz and their count in st->n_rz).
template <class T>
void vcycle_part(Hier &h, const double *y0, double *z0, PcgState *st, bool dot, bool head, bool tail, hipStream_t s) {
    const int L = h.nlev - 1;
    if (L == 0) {  // one level: direct solve (FP64)
        if (head) coarse_solve<double>(h.nL, h.cinv, y0, z0, st, s);
        if (tail && dot) dot_partials(h.nL, y0, z0, h.prz, st_count(st, offsetof(PcgState, n_rz)), st, s);
        return;
    }
    // the level-0 iterate ends up in s or t depending on nu_pre
    T *s0 = (h.lev[0].fsai || h.prm.nu_pre % 2 == 1) ? VT<T>::s(h.lev[0]) : VT<T>::t(h.lev[0]);
    if (head) {
        T *sv[CAMG_MAX_LEVELS] = {};
        for (int l = 0; l < L; ++l) {
            Level &Lv = h.lev[l];
            if (l == 0) sv[0] = smooth_pre<T, double>(h, Lv, y0, st, s);
            else sv[l] = smooth_pre<T, T>(h, Lv, VT<T>::y(Lv), st, s);
            vc_restrict<T>(Lv.R, Lv.cR, VT<T>::r(Lv), VT<T>::y(h.lev[l + 1]), st, s);
        }
        coarse_solve<T>(h.nL, h.cinv, VT<T>::y(h.lev[L]), VT<T>::z(h.lev[L]), st, s);
        for (int l = L - 1; l >= 0; --l) {
            Level &Lv = h.lev[l];
            vc_prolong<T>(Lv.P, Lv.cP, VT<T>::z(h.lev[l + 1]), sv[l], st, s);
            if (l > 0) smooth_post<T, T, T>(h, Lv, VT<T>::y(Lv), sv[l], VT<T>::z(Lv), false, st, s);
        }
        if (sv[0] != s0) fail(CAMG_E_DEVICE, "internal: unexpected smoothing buffer");
    }
    if (tail) smooth_post<T, double, double>(h, h.lev[0], y0, s0, z0, dot, st, s);
}

void vcycle(Hier &h, const double *y0, double *z0, PcgState *st, bool dot, bool head, bool tail, hipStream_t s) {
    if (h.prm.precision == CAMG_MIXED_FP32) vcycle_part<float>(h, y0, z0, st, dot, head, tail, s);
    else vcycle_part<double>(h, y0, z0, st, dot, head, tail, s);
}

// ---------------------------------------------------------------- PCG
void ensure_hist(Hier &h, int cap) {
    if (h.dhist_cap >= cap) return;
    h.dhist = h.pool.alloc<double>(cap);
    h.dhist_cap = cap;
    h.graph_ok = false;
}

// One PCG iteration of parity `par` (p[par] holds the previous direction)
// in three segments: (0) stopping test and the V-cycle up to the level-0
// prolongation, (1) level-0 post-smoothing with the r.z partials, (2) new
// direction with q = A p, then the x / r update.
void enqueue_segment(Hier &h, int par, int seg, hipStream_t s) {
    const Csr &A = h.lev[0].A;
    if (seg == 0) {
        pcg_check(h.pr2, h.st, h.dhist, h.dhist_cap, h.hflag_dev, s);
        vcycle(h, h.r, h.z, h.st, true, true, false, s);
    } else if (seg == 1) {
        vcycle(h, h.r, h.z, h.st, true, false, true, s);
    } else {
        pcg_dir(A, h.lev[0].cA, h.z, h.p[par], h.p[1 - par], h.q, h.prz, h.ppq, h.st, s);
        pcg_update(A.nr, h.p[1 - par], h.q, h.x, h.r, h.ppq, h.pr2, h.st, h.hflag_dev, s);
    }
}

void destroy_graphs(Hier &h) {
    for (int k = 0; k < 4; ++k)
        for (int p = 0; p < 2; ++p) {
            if (h.gexec[k][p]) (void)hipGraphExecDestroy(h.gexec[k][p]);
            if (h.graph[k][p]) (void)hipGraphDestroy(h.graph[k][p]);
            h.gexec[k][p] = nullptr;
            h.graph[k][p] = nullptr;
        }
    h.graph_ok = false;
}

// Capture graphs of the iteration (their kernel arguments only name buffers
// the handle owns, so they stay valid across solves): without timing one
// graph per parity, and one of two iterations (parity 0 then 1: the device
// leaves a gap of some 13 us between two graph launches, paid once per two
// iterations then); with timing, segments 0 and 2 as graphs, so that the
// level-0 post-smoothing kernel can be launched between two stream events.
void build_graphs(Hier &h) {
    destroy_graphs(h);
    if (!h.cap_stream) HIPC(hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking));
    auto capture = [&](int slot, int par, int s0, int s1, bool two = false) {
        HIPC(hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal));
        try {
            for (int seg = s0; seg <= s1; ++seg) enqueue_segment(h, par, seg, h.cap_stream);
            if (two)
                for (int seg = s0; seg <= s1; ++seg) enqueue_segment(h, 1 - par, seg, h.cap_stream);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(h.cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        HIPC(hipStreamEndCapture(h.cap_stream, &h.graph[slot][par]));
        HIPC(hipGraphInstantiate(&h.gexec[slot][par], h.graph[slot][par], nullptr, nullptr, 0));
    };
    for (int p = 0; p < 2; ++p) {
        capture(0, p, 0, 2);
        if (h.prof) {  // timed iterations: the level-0 post-smoothing kernel between two events
            capture(1, p, 0, 0);
            capture(2, p, 2, 2);
        }
    }
    capture(3, 0, 0, 2, true);
    h.graph_ok = true;
    h.graph_prof = h.prof;
}

void launch_iteration(Hier &h, int par, bool timed, hipStream_t s) {
    const bool g = h.use_graph && h.graph_ok;
    if (g && !timed) {
        HIPC(hipGraphLaunch(h.gexec[0][par], s));
        return;
    }
    if (g) HIPC(hipGraphLaunch(h.gexec[1][par], s));
    else enqueue_segment(h, par, 0, s);
    // with Jacobi the segment is the one post-smoothing kernel, whose launch
    // records the events itself; the two FSAI kernels sit between stream events
    const bool one = !h.lev[0].fsai;
    if (timed && one) time_next_row_launch(h.pev[par][0], h.pev[par][1]);
    if (timed && !one) HIPC(hipEventRecord(h.pev[par][0], s));
    enqueue_segment(h, par, 1, s);
    if (timed && one && cancel_row_launch_timing()) {  // no row kernel in the segment
        HIPC(hipEventRecord(h.pev[par][0], s));
        HIPC(hipEventRecord(h.pev[par][1], s));
    }
    if (timed && !one) HIPC(hipEventRecord(h.pev[par][1], s));
    if (g) HIPC(hipGraphLaunch(h.gexec[2][par], s));
    else enqueue_segment(h, par, 2, s);
}

// PCG iterations k = k0 .. max_iter-1 (fewer if the stopping test or a
// breakdown ends them).  The host polls a host-mapped flag one iteration
// behind the device, so the queue never runs dry.  With timing on, the
// level-0 post-smoothing time of iteration k is appended to `times`.
void run_iterations(Hier &h, int k0, std::vector<std::pair<int, float>> &times, hipStream_t s) {
    const int max_iter = h.prm.max_iter;
    if (h.use_graph && (!h.graph_ok || h.graph_prof != h.prof)) {
        try {
            build_graphs(h);
        } catch (const Error &) {
            destroy_graphs(h);
            h.use_graph = false;
        }
    }
    hipEvent_t ev[2];
    HIPC(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    HIPC(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
    } eg{ev};
    // with timing on, every prof_stride-th iteration is timed (the last of each stride)
    auto timed = [&](int k) { return h.prof && (k % h.prof_stride) == h.prof_stride - 1; };
    auto collect = [&](int k) {
        if (!timed(k)) return;
        float ms = 0.f;
        HIPC(hipEventElapsedTime(&ms, h.pev[k & 1][0], h.pev[k & 1][1]));
        times.emplace_back(k, ms);
    };
    volatile int32_t *flag = h.hflag;
    flag[0] = 0;
    int last = -1;
    // launches alternate between the two events; pk/pn: the first iteration
    // and the number of iterations of the previous launch; iterations below
    // `seen` have had their timings collected
    int cur = 0, pk = -1, pn = 0, seen = k0;
    for (int k = k0; k < max_iter;) {
        const int par = k & 1;
        int nk = 1;
        if (h.use_graph && h.graph_ok && par == 0 && k + 1 < max_iter && !timed(k) && !timed(k + 1)) {
            HIPC(hipGraphLaunch(h.gexec[3][0], s));
            nk = 2;
        } else {
            launch_iteration(h, par, timed(k), s);
        }
        HIPC(hipEventRecord(ev[cur], s));
        last = k + nk - 1;
        if (pk >= 0) {
            HIPC(hipEventSynchronize(ev[1 - cur]));
            for (int j = pk; j < pk + pn; ++j) collect(j);
            seen = pk + pn;
            if (flag[0]) break;
        }
        pk = k;
        pn = nk;
        cur = 1 - cur;
        k += nk;
    }
    // the stopping test for the last residual formed
    pcg_check(h.pr2, h.st, h.dhist, h.dhist_cap, h.hflag_dev, s);
    HIPC(hipStreamSynchronize(s));
    for (int j = seen; j <= last; ++j) collect(j);
}

double true_relres_of(Hier &h, const double *b, const double *x, double bnorm, double *r_out, hipStream_t s) {
    const Csr &A = h.lev[0].A;
    double *part = r_out ? h.pr2 : h.ptmp;
    int32_t *nout = r_out ? st_count(h.st, offsetof(PcgState, n_r2)) : nullptr;
    const int np = residual_norm(A, h.lev[0].cA, b, x, r_out, part, nout, s);
    sum_to(part, np, h.sc, s);
    const double t2 = read1(h.sc, s);
    return bnorm > 0.0 ? std::sqrt(t2) / bnorm : 0.0;
}

camg_status solve_dev(Hier &h, const double *b, double rtol, double *x, int32_t *iters, double *hist, int hist_cap,
                      double *true_relres, hipStream_t s) {
    const Csr &A = h.lev[0].A;
    const int n = A.nr;
    ensure_hist(h, h.prm.max_iter + 2);
    std::vector<std::pair<int, float>> times;
    pcg_init(n, b, h.x, h.r, h.p[0], rtol, h.pr2, h.st, s);
    run_iterations(h, 0, times, s);
    PcgState st = read1(h.st, s);
    double rel = -1.0;
    // mixed precision: if the recursive residual met the test but the true
    // one does not, restart from r = b - A x (at most twice)
    if (h.prm.precision == CAMG_MIXED_FP32 && rtol > 0.0) {
        for (int rep = 0; rep < 2 && st.done && st.status == 0; ++rep) {
            rel = true_relres_of(h, b, h.x, st.bnorm, nullptr, s);
            if (rel < rtol || st.iter >= h.prm.max_iter) break;
            true_relres_of(h, b, h.x, st.bnorm, h.r, s);
            pcg_restart(h.st, s);
            run_iterations(h, st.iter, times, s);
            st = read1(h.st, s);
            rel = -1.0;
        }
    }
    // mixed precision promises the true residual: after the restarts, a
    // recursive stop whose true residual still fails is an accuracy warning
    bool inaccurate = false;
    if (h.prm.precision == CAMG_MIXED_FP32 && rtol > 0.0 && st.done && st.status == 0 && st.bnorm > 0.0) {
        if (rel < 0.0) rel = true_relres_of(h, b, h.x, st.bnorm, nullptr, s);
        inaccurate = rel >= rtol;
    }
    // launches after convergence return at once: keep the iterations that ran
    for (const auto &t : times)
        if (t.first < st.iter) {
            h.prof_ms += t.second;
            h.prof_launches += 1;
        }
    HIPC(hipMemcpyAsync(x, h.x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
    const int it = st.iter;
    if (iters) *iters = it;
    if (hist && hist_cap > 0) {
        const int m = std::min(hist_cap, it + 1);
        HIPC(hipMemcpyAsync(hist, h.dhist, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    }
    if (true_relres) *true_relres = rel >= 0.0 ? rel : true_relres_of(h, b, h.x, st.bnorm, nullptr, s);
    HIPC(hipStreamSynchronize(s));
    if (st.status == (int32_t)CAMG_E_BREAKDOWN) {
        g_last_error = "CG breakdown: p.Ap <= 0 or r.z <= 0";
        return CAMG_E_BREAKDOWN;
    }
    if (!st.done) {
        g_last_error = "max_iter reached";
        return CAMG_E_MAXIT;
    }
    if (inaccurate) {
        g_last_error = "true residual above rtol after two restarts (mixed precision)";
        return CAMG_E_ACCURACY;
    }
    return CAMG_OK;
}

Hier *as_hier(camg_handle h) {
    if (!h) fail(CAMG_E_ARG, "null handle");
    return reinterpret_cast<Hier *>(h);
}

}  // namespace
}  // namespace camg

using namespace camg;

struct camg_hier : public camg::Hier {};

extern "C" {

int32_t camg_abi_version(void) { return CAMG_ABI_VERSION; }

const char *camg_status_str(camg_status s) {
    switch (s) {
    case CAMG_OK: return "ok";
    case CAMG_E_MAXIT: return "maximum number of iterations reached";
    case CAMG_E_ACCURACY: return "true residual above the tolerance (mixed precision)";
    case CAMG_E_ARG: return "invalid argument";
    case CAMG_E_CSR: return "malformed or unsupported CSR matrix";
    case CAMG_E_NOT_SPD: return "matrix is not symmetric positive definite";
    case CAMG_E_BREAKDOWN: return "conjugate gradient breakdown";
    case CAMG_E_COARSE: return "coarsening stalled";
    case CAMG_E_NOMEM: return "out of memory";
    case CAMG_E_DEVICE: return "HIP runtime error";
    case CAMG_E_BUSY: return "handle busy";
    }
    return "unknown status";
}

const char *camg_last_error(void) { return camg::g_last_error.c_str(); }

void camg_params_default(camg_params *p) {
    if (!p) return;
    p->theta = 0.25;
    p->seed = 0;
    p->nu_pre = 1;
    p->nu_post = 1;
    p->omega = 0.0;
    p->max_levels = 25;
    p->max_coarse = 256;
    p->precision = CAMG_FP64;
    p->max_iter = 1000;
    p->smoother = CAMG_SMOOTH_JACOBI;
    p->interp = CAMG_INTERP_DIRECT;
    p->rap_chunk = 0;
    p->bamg_lmin = 1;
    p->bamg_lmax = 2;
    p->bamg_eps = 1e-3;
    p->bamg_mu = 10.0;
    p->psmooth = 0;
    p->pfilter = 1.0;
    p->srqm_iters = 0;
    p->afsai_steps = 10;
    p->afsai_step = 2;
    p->afsai_eps = 0.01;
}

static camg_status setup_common(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nt,
                                const double *V, const camg_params *params, void *stream, bool host_in,
                                camg_handle *out) {
    return guarded([&] {
        if (!out) fail(CAMG_E_ARG, "null output handle");
        *out = nullptr;
        if (n < 1 || !rp || !ci || !v) fail(CAMG_E_ARG, "n < 1 or null CSR array");
        std::unique_ptr<camg_hier> h(new camg_hier());
        if (params) h->prm = *params;
        else camg_params_default(&h->prm);
        check_params(h->prm);
        if (h->prm.interp == CAMG_INTERP_BAMG && (nt < 1 || nt > 8 || !V))
            fail(CAMG_E_ARG, "BAMG interpolation needs a test space of 1 to 8 vectors (camg_setup_tv)");
        HIPC(hipGetDevice(&h->device));
        build_hierarchy(*h, n, rp, ci, v, nt, V, host_in, (hipStream_t)stream);
        *out = h.release();
    });
}

camg_status camg_setup(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                       const camg_params *params, camg_handle *out) {
    if (n >= 1 && row_ptr && (row_ptr[0] != 0 || row_ptr[n] < 0)) {
        g_last_error = "row pointer is not 0-based";
        if (out) *out = nullptr;
        return CAMG_E_CSR;
    }
    return setup_common(n, row_ptr, col_idx, val, 0, nullptr, params, nullptr, true, out);
}

camg_status camg_setup_dev(int32_t n, const int32_t *d_row_ptr, const int32_t *d_col_idx, const double *d_val,
                           const camg_params *params, void *hip_stream, camg_handle *out) {
    return setup_common(n, d_row_ptr, d_col_idx, d_val, 0, nullptr, params, hip_stream, false, out);
}

camg_status camg_setup_tv(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val, int32_t nt,
                          const double *V, const camg_params *params, camg_handle *out) {
    if (n >= 1 && row_ptr && (row_ptr[0] != 0 || row_ptr[n] < 0)) {
        g_last_error = "row pointer is not 0-based";
        if (out) *out = nullptr;
        return CAMG_E_CSR;
    }
    return setup_common(n, row_ptr, col_idx, val, nt, V, params, nullptr, true, out);
}

camg_status camg_setup_tv_dev(int32_t n, const int32_t *d_row_ptr, const int32_t *d_col_idx, const double *d_val,
                              int32_t nt, const double *d_V, const camg_params *params, void *hip_stream,
                              camg_handle *out) {
    return setup_common(n, d_row_ptr, d_col_idx, d_val, nt, d_V, params, hip_stream, false, out);
}

camg_status camg_solve_dev(camg_handle hh, const double *d_b, double rtol, double *d_x, int32_t *iters,
                           double *hist, int32_t hist_cap, double *true_relres, void *hip_stream) {
    camg_status ret = CAMG_OK;
    camg_status st = guarded([&] {
        Hier *h = as_hier(hh);
        if (!d_b || !d_x) fail(CAMG_E_ARG, "null vector");
        if (!std::isfinite(rtol)) fail(CAMG_E_ARG, "rtol must be finite");
        BusyGuard g(h);
        HIPC(hipSetDevice(h->device));
        ret = solve_dev(*h, d_b, rtol, d_x, iters, hist, hist_cap, true_relres, (hipStream_t)hip_stream);
    });
    return st != CAMG_OK ? st : ret;
}

camg_status camg_solve(camg_handle hh, const double *b, double rtol, double *x, int32_t *iters, double *hist,
                       int32_t hist_cap, double *true_relres) {
    camg_status ret = CAMG_OK;
    camg_status st = guarded([&] {
        Hier *h = as_hier(hh);
        if (!b || !x) fail(CAMG_E_ARG, "null vector");
        if (!std::isfinite(rtol)) fail(CAMG_E_ARG, "rtol must be finite");
        BusyGuard g(h);
        HIPC(hipSetDevice(h->device));
        const int n = h->lev[0].A.nr;
        Pool io((hipStream_t) nullptr);
        double *db = io.alloc<double>(n), *dx = io.alloc<double>(n);
        HIPC(hipMemcpy(db, b, sizeof(double) * n, hipMemcpyHostToDevice));
        ret = solve_dev(*h, db, rtol, dx, iters, hist, hist_cap, true_relres, nullptr);
        HIPC(hipMemcpy(x, dx, sizeof(double) * n, hipMemcpyDeviceToHost));
    });
    return st != CAMG_OK ? st : ret;
}

camg_status camg_vcycle_dev(camg_handle hh, const double *d_y, double *d_z, void *hip_stream) {
    return guarded([&] {
        Hier *h = as_hier(hh);
        if (!d_y || !d_z) fail(CAMG_E_ARG, "null vector");
        BusyGuard g(h);
        HIPC(hipSetDevice(h->device));
        vcycle(*h, d_y, d_z, nullptr, false, true, true, (hipStream_t)hip_stream);
        HIPC(hipStreamSynchronize((hipStream_t)hip_stream));
    });
}

camg_status camg_info(camg_handle hh, camg_info_t *info) {
    return guarded([&] {
        Hier *h = as_hier(hh);
        if (!info) fail(CAMG_E_ARG, "null info");
        std::memset(info, 0, sizeof(*info));
        info->levels = h->nlev;
        double sn = 0, sz = 0;
        for (int l = 0; l < h->nlev; ++l) {
            const Level &L = h->lev[l];
            info->n[l] = L.A.nr;
            info->nnz[l] = L.A.nnz;
            info->nnz_p[l] = l < h->nlev - 1 ? L.P.nnz : 0;
            info->pmis_rounds[l] = L.rounds;
            info->omega[l] = L.omega;
            sn += L.A.nr;
            sz += (double)L.A.nnz;
        }
        info->grid_complexity = sn / h->lev[0].A.nr;
        info->operator_complexity = sz / (double)h->lev[0].A.nnz;
        info->device_bytes = h->pool.bytes;
        info->setup_ms = h->setup_ms;
        info->precision = h->prm.precision;
        for (int k = 0; k < 8; ++k) info->setup_phase_ms[k] = h->phase_ms[k];
        info->compact_cols = 0;
        for (int l = 0; l < h->nlev && l < 6; ++l) {
            const Level &L = h->lev[l];
            const RowCfg *cs[5] = {&L.cA, &L.cP, &L.cR, &L.cG, &L.cGt};
            for (int k = 0; k < 5; ++k)
                if (cs[k]->off) info->compact_cols |= 1 << (5 * l + k);
        }
    });
}

camg_status camg_level_sizes(camg_handle hh, int32_t l, int32_t *n, int64_t *nnz_a, int64_t *nnz_p, int32_t *nc) {
    return guarded([&] {
        Hier *h = as_hier(hh);
        if (l < 0 || l >= h->nlev) fail(CAMG_E_ARG, "level out of range");
        const Level &L = h->lev[l];
        const bool last = l == h->nlev - 1;
        if (n) *n = L.A.nr;
        if (nnz_a) *nnz_a = L.A.nnz;
        if (nnz_p) *nnz_p = last ? 0 : L.P.nnz;
        if (nc) *nc = last ? 0 : L.P.nc;
    });
}

static void copy_csr_out(const Csr &M, void *a, void *b, void *c) {
    if (a) HIPC(hipMemcpy(a, M.rp, sizeof(int32_t) * ((size_t)M.nr + 1), hipMemcpyDeviceToHost));
    if (b && M.nnz) HIPC(hipMemcpy(b, M.ci, sizeof(int32_t) * (size_t)M.nnz, hipMemcpyDeviceToHost));
    if (c && M.nnz) HIPC(hipMemcpy(c, M.v, sizeof(double) * (size_t)M.nnz, hipMemcpyDeviceToHost));
}

camg_status camg_export_level(camg_handle hh, int32_t l, int32_t what, void *a, void *b, void *c) {
    return guarded([&] {
        Hier *h = as_hier(hh);
        if (l < 0 || l >= h->nlev) fail(CAMG_E_ARG, "level out of range");
        BusyGuard g(h);
        HIPC(hipSetDevice(h->device));
        const Level &L = h->lev[l];
        const bool last = l == h->nlev - 1;
        const int n = L.A.nr;
        if (what != CAMG_X_A && what != CAMG_X_COARSE_INV && last) fail(CAMG_E_ARG, "no such data on the last level");
        if (!a) fail(CAMG_E_ARG, "null output");
        switch (what) {
        case CAMG_X_A: copy_csr_out(L.A, a, b, c); break;
        case CAMG_X_P: copy_csr_out(L.P, a, b, c); break;
        case CAMG_X_R: copy_csr_out(L.R, a, b, c); break;
        case CAMG_X_CF: HIPC(hipMemcpy(a, L.cf, (size_t)n, hipMemcpyDeviceToHost)); break;
        case CAMG_X_STRONG: HIPC(hipMemcpy(a, L.strong, (size_t)L.A.nnz, hipMemcpyDeviceToHost)); break;
        case CAMG_X_DINV: HIPC(hipMemcpy(a, L.dinv, sizeof(double) * n, hipMemcpyDeviceToHost)); break;
        case CAMG_X_OMEGA: std::memcpy(a, &L.omega, sizeof(double)); break;
        case CAMG_X_STCNT: HIPC(hipMemcpy(a, L.stcnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost)); break;
        case CAMG_X_G:
            if (!L.G.rp) fail(CAMG_E_ARG, "the handle does not use the FSAI smoother");
            copy_csr_out(L.G, a, b, c);
            break;
        case CAMG_X_COARSE_INV:
            if (!last) fail(CAMG_E_ARG, "the dense inverse exists on the last level only");
            HIPC(hipMemcpy(a, h->cinv, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToHost));
            break;
        default: fail(CAMG_E_ARG, "unknown export selector");
        }
    });
}

camg_status camg_galerkin(int32_t n, const int32_t *a_rp, const int32_t *a_ci, const double *a_val, int32_t nc,
                          const int32_t *p_rp, const int32_t *p_ci, const double *p_val, int32_t **c_rp,
                          int32_t **c_ci, double **c_val, int64_t *nnz_out) {
    return guarded([&] {
        if (n < 1 || nc < 0 || !a_rp || !a_ci || !a_val || !p_rp || !p_ci || !p_val || !c_rp || !c_ci || !c_val)
            fail(CAMG_E_ARG, "bad argument");
        hipStream_t s = nullptr;
        Pool tmp(s), outp(s);
        auto up = [&](Csr &M, int nr, int ncol, const int32_t *rp, const int32_t *ci, const double *v) {
            M.nr = nr;
            M.nc = ncol;
            M.nnz = rp[nr];
            M.rp = tmp.alloc<int32_t>((size_t)nr + 1);
            M.ci = tmp.alloc<int32_t>(padded(M.nnz));
            M.v = tmp.alloc<double>(padded(M.nnz));
            HIPC(hipMemcpy(M.rp, rp, sizeof(int32_t) * ((size_t)nr + 1), hipMemcpyHostToDevice));
            if (M.nnz) {
                HIPC(hipMemcpy(M.ci, ci, sizeof(int32_t) * (size_t)M.nnz, hipMemcpyHostToDevice));
                HIPC(hipMemcpy(M.v, v, sizeof(double) * (size_t)M.nnz, hipMemcpyHostToDevice));
            }
        };
        Csr A, P, R, AP, C;
        up(A, n, n, a_rp, a_ci, a_val);
        up(P, n, nc, p_rp, p_ci, p_val);
        R.nr = nc;
        R.nc = n;
        R.nnz = P.nnz;
        int32_t *ccnt = tmp.alloc<int32_t>(std::max(nc, 1));
        column_counts(P, ccnt, s);
        int64_t *rrp64 = tmp.alloc<int64_t>((size_t)nc + 1);
        scan_i32_to_i64(ccnt, rrp64, nc, tmp, s);
        R.rp = tmp.alloc<int32_t>((size_t)nc + 1);
        narrow_i64(rrp64, R.rp, nc, s);
        R.ci = tmp.alloc<int32_t>(padded(R.nnz));
        R.v = tmp.alloc<double>(padded(R.nnz));
        transpose_csr(P, R, tmp, s);
        spgemm(A, P, AP, tmp, tmp, s);
        spgemm(R, AP, C, outp, tmp, s);
        HIPC(hipDeviceSynchronize());
        *c_rp = (int32_t *)std::malloc(sizeof(int32_t) * ((size_t)nc + 1));
        *c_ci = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(C.nnz, 1));
        *c_val = (double *)std::malloc(sizeof(double) * (size_t)std::max<int64_t>(C.nnz, 1));
        if (!*c_rp || !*c_ci || !*c_val) fail(CAMG_E_NOMEM, "host allocation failed");
        copy_csr_out(C, *c_rp, *c_ci, *c_val);
        if (nnz_out) *nnz_out = C.nnz;
    });
}

void camg_free_host(void *p) { std::free(p); }

camg_status camg_destroy(camg_handle hh) {
    if (!hh) return CAMG_OK;
    return guarded([&] {
        Hier *h = as_hier(hh);
        (void)hipSetDevice(h->device);
        (void)hipDeviceSynchronize();
        if (h->hflag) (void)hipHostFree(h->hflag);
        for (auto &pp : h->pev)
            for (auto &e : pp)
                if (e) (void)hipEventDestroy(e);
        destroy_graphs(*h);
        if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
        for (Engine *e : h->engines) engine_destroy(e);
        h->engines.clear();
        delete static_cast<camg_hier *>(hh);
    });
}

camg_status camg_profile(camg_handle hh, int32_t enable, double *total_ms, int64_t *launches) {
    return guarded([&] {
        Hier *h = as_hier(hh);
        BusyGuard g(h);
        HIPC(hipSetDevice(h->device));
        if (total_ms) *total_ms = h->prof_ms;
        if (launches) *launches = h->prof_launches;
        h->prof_ms = 0.0;
        h->prof_launches = 0;
        if (enable < 0) fail(CAMG_E_ARG, "enable must be >= 0");
        const bool on = enable != 0;
        if (on && !h->pev[0][0])
            for (auto &pp : h->pev)
                for (auto &e : pp) HIPC(hipEventCreate(&e));
        h->prof = on;
        h->prof_stride = on ? enable : 1;
    });
}

camg_status camg_set_option(camg_handle hh, int32_t option, int64_t value) {
    return guarded([&] {
        Hier *h = as_hier(hh);
        BusyGuard g(h);
        switch (option) {
        case CAMG_OPT_GRAPH:
            h->use_graph = value != 0;
            h->graph_ok = false;
            break;
        case CAMG_OPT_AUTOTUNE:
            h->autotune = value != 0;
            break;
        case CAMG_OPT_COMPACT_COLS:
            h->compact_cols = value != 0;
            for (Level &L : h->lev)
                for (RowCfg *c : {&L.cA, &L.cP, &L.cR, &L.cG, &L.cGt}) c->use_off = h->compact_cols && c->off;
            h->graph_ok = false;  // captured launches hold the old arguments
            break;
        default: fail(CAMG_E_ARG, "unknown option");
        }
    });
}

static int pow2_at_least(int k) {
    int K = 1;
    while (K < k) K <<= 1;
    return K;
}

static Engine *engine_for(Hier *h, int K, hipStream_t s) {
    for (Engine *e : h->engines)
        if (engine_slots(*e) == K) return e;
    Engine *e = engine_create(*h, K, h->prm.max_iter + 2, s);
    h->engines.push_back(e);
    return e;
}

camg_status camg_solve_multi_dev(camg_handle hh, int32_t k, const double *d_B, double rtol, double *d_X,
                                 int32_t *iters, double *hist, int32_t hist_cap, double *true_relres,
                                 void *hip_stream) {
    camg_status worst = CAMG_OK;
    camg_status st = guarded([&] {
        Hier *h = as_hier(hh);
        if (k < 1 || !d_B || !d_X) fail(CAMG_E_ARG, "k < 1 or null block");
        if (!std::isfinite(rtol)) fail(CAMG_E_ARG, "rtol must be finite");
        BusyGuard g(h);
        HIPC(hipSetDevice(h->device));
        hipStream_t s = (hipStream_t)hip_stream;
        const int K = pow2_at_least(std::min<int>(k, kMaxSlots));
        Engine *E = engine_for(h, K, s);
        std::vector<int32_t> it(K), dn(K), stt(K);
        std::vector<double> rel(K);
        for (int c0 = 0; c0 < k; c0 += K) {
            const int m = std::min(K, k - c0);
            engine_start(*E, 0, m, d_B + c0, k, rtol, h->prm.max_iter, s);
            engine_step(*E, h->prm.max_iter + 1, s);
            engine_slot_state(*E, it.data(), dn.data(), stt.data(), s);
            if (h->prm.precision == CAMG_MIXED_FP32 && rtol > 0.0) {
                for (int rep = 0; rep < 2; ++rep) {
                    engine_true_res(*E, rel.data(), s);
                    unsigned long long mask = 0;
                    for (int c = 0; c < m; ++c)
                        if (stt[c] == 0 && rel[c] >= rtol && it[c] < h->prm.max_iter) mask |= 1ull << c;
                    if (!mask) break;
                    engine_replace(*E, mask, s);
                    engine_step(*E, h->prm.max_iter + 1, s);
                    engine_slot_state(*E, it.data(), dn.data(), stt.data(), s);
                }
            }
            engine_true_res(*E, rel.data(), s);
            engine_copy_x(*E, 0, m, d_X + c0, k, s);
            for (int c = 0; c < m; ++c) {
                if (iters) iters[c0 + c] = it[c];
                if (true_relres) true_relres[c0 + c] = rel[c];
                if (hist && hist_cap > 0) engine_hist(*E, c, hist + (size_t)(c0 + c) * hist_cap, hist_cap, it[c] + 1, s);
                camg_status cs = (camg_status)stt[c];
                if (cs == CAMG_OK && h->prm.precision == CAMG_MIXED_FP32 && rtol > 0.0 && rel[c] >= rtol)
                    cs = CAMG_E_ACCURACY;
                worst = worse_status(worst, cs);
            }
            engine_release(*E, 0, m, s);
        }
        HIPC(hipStreamSynchronize(s));
    });
    if (st != CAMG_OK) return st;
    if (worst == CAMG_E_BREAKDOWN) camg::g_last_error = "CG breakdown in at least one column";
    if (worst == CAMG_E_MAXIT) camg::g_last_error = "max_iter reached in at least one column";
    if (worst == CAMG_E_ACCURACY)
        camg::g_last_error = "true residual above rtol after two restarts in at least one column";
    return worst;
}

// ---------------------------------------------------------------- engine (serving) API
struct camg_engine {
    Engine *e = nullptr;
    Hier *h = nullptr;
    hipStream_t s = nullptr;
};

camg_status camg_engine_footprint(camg_handle hh, int32_t slots, int64_t *bytes) {
    return guarded([&] {
        Hier *h = as_hier(hh);
        if (!bytes || slots < 1 || slots > kMaxSlots) fail(CAMG_E_ARG, "bad argument");
        *bytes = engine_footprint(*h, pow2_at_least(slots));
    });
}

camg_status camg_engine_create(camg_handle hh, int32_t slots, int32_t hist_cap, void *hip_stream, camg_engine_t *out) {
    return guarded([&] {
        Hier *h = as_hier(hh);
        if (!out) fail(CAMG_E_ARG, "null output");
        *out = nullptr;
        if (slots < 1 || slots > kMaxSlots || (slots & (slots - 1)))
            fail(CAMG_E_ARG, "slots must be a power of two in [1, 64]");
        HIPC(hipSetDevice(h->device));
        std::unique_ptr<camg_engine> ce(new camg_engine());
        ce->h = h;
        ce->s = (hipStream_t)hip_stream;
        ce->e = engine_create(*h, slots, std::max(hist_cap, 1), ce->s);
        *out = ce.release();
    });
}

camg_status camg_engine_start(camg_engine_t ce, int32_t slot0, int32_t m, const double *d_B, int32_t ldb, double rtol,
                              int32_t max_iter) {
    return guarded([&] {
        if (!ce || !d_B || ldb < m) fail(CAMG_E_ARG, "bad argument");
        HIPC(hipSetDevice(ce->h->device));
        engine_start(*ce->e, slot0, m, d_B, ldb, rtol, max_iter, ce->s);
    });
}

camg_status camg_engine_step(camg_engine_t ce, int32_t max_steps, int32_t *running) {
    return guarded([&] {
        if (!ce || max_steps < 1) fail(CAMG_E_ARG, "bad argument");
        HIPC(hipSetDevice(ce->h->device));
        const int r = engine_step(*ce->e, max_steps, ce->s);
        if (running) *running = r;
    });
}

camg_status camg_engine_state(camg_engine_t ce, int32_t *iters, int32_t *done, int32_t *status) {
    return guarded([&] {
        if (!ce) fail(CAMG_E_ARG, "null engine");
        HIPC(hipSetDevice(ce->h->device));
        engine_slot_state(*ce->e, iters, done, status, ce->s);
    });
}

camg_status camg_engine_finish(camg_engine_t ce, int32_t slot0, int32_t m, double *d_X, int32_t ldx,
                               double *true_relres) {
    return guarded([&] {
        if (!ce || !d_X || ldx < m || slot0 < 0 || m < 1 || slot0 + m > engine_slots(*ce->e))
            fail(CAMG_E_ARG, "bad argument");
        HIPC(hipSetDevice(ce->h->device));
        if (true_relres) {
            double rel[kMaxSlots];
            engine_true_res(*ce->e, rel, ce->s);
            for (int c = 0; c < m; ++c) true_relres[c] = rel[slot0 + c];
        }
        engine_copy_x(*ce->e, slot0, m, d_X, ldx, ce->s);
        engine_release(*ce->e, slot0, m, ce->s);
    });
}

camg_status camg_engine_destroy(camg_engine_t ce) {
    if (!ce) return CAMG_OK;
    return guarded([&] {
        (void)hipSetDevice(ce->h->device);
        (void)hipStreamSynchronize(ce->s);
        engine_destroy(ce->e);
        delete ce;
    });
}

// ---------------------------------------------------------------- many small systems
namespace {
camg_status batch_entry(int32_t count, const camg_handle *hs, const double *const *d_b, double *const *d_x,
                        double rtol, int32_t *iters, double *true_relres, int32_t *status, void *hip_stream,
                        bool no_alloc) {
    return guarded([&] {
        if (count < 1 || !hs || !d_b || !d_x) fail(CAMG_E_ARG, "count < 1 or null array");
        if (no_alloc && count > CAMG_NOALLOC_MAX_SYSTEMS)
            fail(CAMG_E_ARG, "more systems than the allocation-free batch holds (CAMG_NOALLOC_MAX_SYSTEMS)");
        if (!std::isfinite(rtol)) fail(CAMG_E_ARG, "rtol must be finite");
        std::vector<Hier *> v(count);
        std::vector<std::unique_ptr<BusyGuard>> guards;
        for (int k = 0; k < count; ++k) {
            v[k] = as_hier(hs[k]);
            if (!d_b[k] || !d_x[k]) fail(CAMG_E_ARG, "null vector");
            guards.emplace_back(new BusyGuard(v[k]));  // also rejects a handle listed twice
        }
        HIPC(hipSetDevice(v[0]->device));
        solve_batch(v, d_b, d_x, rtol, iters, true_relres, status, (hipStream_t)hip_stream, no_alloc);
    });
}
}  // namespace

camg_status camg_solve_batch_dev(int32_t count, const camg_handle *hs, const double *const *d_b, double *const *d_x,
                                 double rtol, int32_t *iters, double *true_relres, int32_t *status,
                                 void *hip_stream) {
    return batch_entry(count, hs, d_b, d_x, rtol, iters, true_relres, status, hip_stream, false);
}

camg_status camg_solve_batch_noalloc_dev(int32_t count, const camg_handle *hs, const double *const *d_b,
                                         double *const *d_x, double rtol, int32_t *iters, double *true_relres,
                                         int32_t *status, void *hip_stream) {
    return batch_entry(count, hs, d_b, d_x, rtol, iters, true_relres, status, hip_stream, true);
}

// ---------------------------------------------------------------- server API
struct camg_server {
    Server *s = nullptr;
    int device = 0;
};

camg_status camg_server_create(int64_t budget_bytes, camg_server_t *out) {
    return guarded([&] {
        if (!out) fail(CAMG_E_ARG, "null output");
        *out = nullptr;
        std::unique_ptr<camg_server> cs(new camg_server());
        HIPC(hipGetDevice(&cs->device));
        cs->s = server_create(budget_bytes);
        *out = cs.release();
    });
}

camg_status camg_server_add(camg_server_t cs, camg_handle hh, int32_t slots, int32_t iters_per_batch,
                            int32_t *system) {
    return guarded([&] {
        if (!cs) fail(CAMG_E_ARG, "null server");
        Hier *h = as_hier(hh);
        if (h->device != cs->device) fail(CAMG_E_ARG, "handle lives on another device");
        HIPC(hipSetDevice(cs->device));
        const int id = server_add(*cs->s, *h, slots, iters_per_batch);
        if (system) *system = id;
    });
}

camg_status camg_server_submit(camg_server_t cs, int32_t system, int32_t k, const double *B, int32_t ldb, double *X,
                               int32_t ldx, double rtol, int32_t max_iter, int64_t tag) {
    return guarded([&] {
        if (!cs) fail(CAMG_E_ARG, "null server");
        HIPC(hipSetDevice(cs->device));
        server_submit(*cs->s, system, k, B, ldb, X, ldx, rtol, max_iter, tag);
    });
}

camg_status camg_server_poll(camg_server_t cs, camg_completion *out, int32_t cap, int32_t *n_out) {
    return guarded([&] {
        if (!cs || cap < 0 || (cap > 0 && !out)) fail(CAMG_E_ARG, "bad argument");
        HIPC(hipSetDevice(cs->device));
        server_poll(*cs->s);
        const int m = server_take(*cs->s, out, cap);
        if (n_out) *n_out = m;
    });
}

camg_status camg_server_stats(camg_server_t cs, int64_t *arena_used, int64_t *arena_size, int32_t *queued,
                              int32_t *busy_slots) {
    return guarded([&] {
        if (!cs) fail(CAMG_E_ARG, "null server");
        server_stats(*cs->s, arena_used, arena_size, queued, busy_slots);
    });
}

camg_status camg_server_destroy(camg_server_t cs) {
    if (!cs) return CAMG_OK;
    return guarded([&] {
        (void)hipSetDevice(cs->device);
        server_destroy(cs->s);
        delete cs;
    });
}

}  // extern "C"
