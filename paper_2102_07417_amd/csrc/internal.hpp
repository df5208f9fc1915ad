// Internal declarations shared by the translation units of libcamg.
// Kernels live next to their host launchers; the driver (camg.hip) only
// calls the launchers declared here.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "camg.h"

namespace camg {

// ---------------------------------------------------------------- errors
struct Error {
    camg_status status;
    std::string msg;
};

[[noreturn]] void fail(camg_status s, const std::string &msg);

// The worse of two per-column outcomes: breakdown, then max_iter, then the
// mixed-precision accuracy warning, then ok.
inline camg_status worse_status(camg_status a, camg_status b) {
    auto rank = [](camg_status s) {
        return s == CAMG_E_BREAKDOWN ? 3 : s == CAMG_E_MAXIT ? 2 : s == CAMG_E_ACCURACY ? 1 : 0;
    };
    return rank(b) > rank(a) ? b : a;
}
void hip_check(hipError_t e, const char *what);
#define HIPC(x) ::camg::hip_check((x), #x)

// ---------------------------------------------------------------- memory
// Device allocations owned by a handle or an engine, or by a set-up scratch
// pool.  Requests are rounded to 256 bytes; small ones are packed into 16 MB
// chunks, large ones get blocks of their own.  A released pool hands its
// blocks to a per-device cache (a scratch pool, constructed with the stream
// its memory is used on, once that stream has drained; an owning pool once
// the blocks' devices have drained, as hipFree would wait for them), and
// later pools take blocks from the cache instead of calling hipMalloc, so
// repeated set-ups and destructions cost no hipMalloc/hipFree (a hipMalloc
// costs tens of microseconds, a hipFree waits for the whole device).  The
// cache keeps at most 4 GiB per device for the life of the process; an
// allocation that fails empties it and tries again.
struct Pool {
    Pool() = default;
    explicit Pool(hipStream_t scratch_stream) : scratch_(true), stream_(scratch_stream) {}
    Pool(const Pool &) = delete;
    Pool &operator=(const Pool &) = delete;
    void *raw(size_t nbytes);
    template <class T> T *alloc(size_t count) { return static_cast<T *>(raw(count * sizeof(T))); }
    void release();
    ~Pool() { release(); }
    int64_t bytes = 0;  // bytes handed out

    struct Block {
        void *p;
        size_t size;
        int device;
    };

  private:
    Block get(size_t size);
    std::vector<Block> blocks_;
    char *cur_ = nullptr;
    size_t left_ = 0;
    bool scratch_ = false;
    hipStream_t stream_ = nullptr;
};

// Column-index and value arrays carry this many elements of padding past
// nnz, so aligned 16-byte vector loads that straddle the end stay inside
// the allocation.
constexpr int64_t kPad = 8;
inline size_t padded(int64_t nnz) { return (size_t)(nnz + kPad); }

struct Csr {
    int32_t nr = 0, nc = 0;
    int64_t nnz = 0;
    int32_t *rp = nullptr;
    int32_t *ci = nullptr;
    double *v = nullptr;
    float *v32 = nullptr;   // FP32 copy of the values (mixed precision)
};

// Launch shape of the row kernels of one matrix (chosen at set-up).
//   tile: tile t holds the rows whose first nonzero lies in [t W, (t+1) W);
//         its products are staged in LDS and `lpr` lanes sum each row;
//         `grid` blocks take `tpb` consecutive tiles each.
//   vector (tile == false): `lpr` lanes walk each row, `rpt` rows per block.
struct RowCfg {
    bool tile = false;
    int lpr = 8;
    int rpt = 0;          // vector mode: rows per block
    int W = 0;            // tile mode: nominal nonzeros per tile
    int tile_nnz = 0;     // LDS entries reserved per block
    int ntiles = 0;
    int grid = 8;
    int tpb = 0;          // consecutive tiles per block
    int maxrow = 0;
    int32_t *tstart = nullptr;  // device: first row of each tile
    // compact column indices (tile mode, when kTileWins windows of 2^kWinBits
    // columns cover every tile): column = tbase[tile * kTileWins + (off >>
    // kWinBits)] + (off & (2^kWinBits - 1)); use_off switches the row kernels
    // between them and the int32 columns (the same results)
    int32_t *tbase = nullptr;
    uint16_t *off = nullptr;
    int off_mode = 0;  // 1: column = tbase[tile * kTileWins] + off; 2: windows as above
    bool use_off = false;
};

struct Level {
    Csr A, P, R;
    double *dinv = nullptr;   // 1 / a_ii
    double *wd = nullptr;     // omega * dinv_i
    float *wd32 = nullptr;
    double *awd = nullptr;    // a_ij * wd_j (pre-smoothing values)
    float *awd32 = nullptr;
    double omega = 0.0;
    int8_t *cf = nullptr;
    uint8_t *strong = nullptr;
    int32_t *stcnt = nullptr;
    int32_t rounds = 0;
    bool fsai = false;  // this level smooths with FSAI (M^{-1} = G^T G), else Jacobi
    // V-cycle work vectors (y: right-hand side, s: smoothed iterate,
    // r: residual, z: result).  Level 0 borrows y and z from PCG.
    double *y = nullptr, *s = nullptr, *r = nullptr, *z = nullptr, *t = nullptr;
    float *y32 = nullptr, *s32 = nullptr, *r32 = nullptr, *z32 = nullptr, *t32 = nullptr;
    RowCfg cA, cP, cR;
    // FSAI smoother (M^{-1} = G^T G), when selected
    Csr G, Gt;
    RowCfg cG, cGt;
};

// Scalars of one PCG recurrence, resident on the device.
// n_r2, n_rz, n_pq: how many per-block partials the last producer of each
// sum wrote (read by the consumer, so launches need no host knowledge).
struct PcgState {
    double rho, rho_old, sigma, alpha, beta, rnorm, bnorm, tol, rtol;
    int32_t iter, done, status, restart;
    int32_t n_r2, n_rz, n_pq, pad;
};

struct Hier {
    int device = 0;
    camg_params prm{};
    std::vector<Level> lev;
    int nlev = 0;
    int nL = 0;             // order of the last level
    double *cinv = nullptr; // dense inverse of the last level (row-major nL x nL)
    float *cinv32 = nullptr;
    Pool pool;              // everything the handle owns
    // PCG work
    double *x = nullptr, *r = nullptr, *z = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr;
    double *pr2 = nullptr;       // per-block partials of ||r||^2
    double *prz = nullptr;       // per-block partials of r.z
    double *ppq = nullptr;       // per-block partials of p.q
    double *ptmp = nullptr;      // per-block partials (true residual)
    double *sc = nullptr;        // device scalars
    PcgState *st = nullptr;      // device state
    double *dhist = nullptr;     // device residual history
    int dhist_cap = 0;
    int32_t *hflag = nullptr;    // host-mapped convergence flags (one per poll slot)
    int32_t *hflag_dev = nullptr;
    std::atomic<int> busy{0};
    double setup_ms = 0.0;
    double phase_ms[8] = {};  // set-up time per phase (camg_info_t.setup_phase_ms)
    // optional timing of the level-0 post-smoothing kernel inside solves
    bool prof = false;
    int prof_stride = 1;  // time every prof_stride-th iteration
    hipEvent_t pev[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [parity][start/end]
    double prof_ms = 0.0;
    int64_t prof_launches = 0;
    // PCG iterations captured as graphs, per parity of the iteration:
    // slot 0 the whole iteration, slots 1 and 2 the parts before and after
    // the level-0 post-smoothing (used while kernel timing is on)
    bool use_graph = true;
    bool autotune = false;  // engines created on the handle tune their row schedules
    bool compact_cols = true;  // row kernels read the 16-bit column differences where built
    bool graph_ok = false;
    bool graph_prof = false;
    hipGraphExec_t gexec[4][2] = {};  // [0] iteration, [1]/[2] its timed segments, [3][0] two iterations
    hipGraph_t graph[4][2] = {};
    hipStream_t cap_stream = nullptr;
    // engines used by camg_solve_multi_dev, by slot count (owned)
    std::vector<struct Engine *> engines;
};

constexpr int kBlock = 256;          // threads per block for row kernels
constexpr int kMaxSlots = 64;        // columns of a multi-RHS engine
constexpr int kMaxGrid = 2048;       // cap on blocks of the reduction kernels
constexpr int kMaxPartials = 8192;   // room for the per-block partials of any producing kernel

// ---------------------------------------------------------------- scan (setup.hip)
// out[0..n] = exclusive prefix sums of in[0..n-1]; out[n] = total.
void scan_i32_to_i64(const int32_t *in, int64_t *out, int n, Pool &tmp, hipStream_t s);
void scan_i64(const int64_t *in, int64_t *out, int n, Pool &tmp, hipStream_t s);
// rp32[i] = (int32) v64[i] for i in [0, n]; host checks the total first.
void narrow_i64(const int64_t *v64, int32_t *rp32, int n, hipStream_t s);

// ---------------------------------------------------------------- set-up kernels (setup.hip)
// flags[0]: row pointer malformed; flags[1]: column out of range / not increasing;
// flags[2]: non-finite value; flags[3]: diagonal missing; flags[4]: asymmetric;
// flags[5]: non-positive diagonal.
void validate_rowptr(int n, int64_t nnz, const int32_t *rp, int32_t *flags, hipStream_t s);
void validate_rows(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, int32_t *flags,
                   unsigned long long *amax_bits, hipStream_t s);
void validate_sym(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v,
                  const unsigned long long *amax_bits, int32_t *flags, int32_t *tpos, hipStream_t s);
void transpose_positions(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, int32_t *tpos, hipStream_t s);
void strength(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *tpos,
              double theta, uint8_t *strong, int32_t *stcnt, hipStream_t s);
// PMIS: *undecided ends positive while undecided points remain, zero once
// every point is C or F
void pmis_init(int n, const int32_t *stcnt, uint64_t seed, int level, uint64_t *u, int8_t *state,
               int32_t *undecided, hipStream_t s);
void pmis_round(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const uint8_t *strong,
                const int32_t *tpos, const int32_t *stcnt, const uint64_t *u, int8_t *state, int8_t *newc,
                int32_t *undecided, hipStream_t s);
void cf_flags(int n, const int8_t *cf, int32_t *isc, hipStream_t s);
void interp_count(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const uint8_t *strong,
                  const int8_t *cf, int32_t *cnt, hipStream_t s);
void interp_fill(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, const uint8_t *strong,
                 const int8_t *cf, const int64_t *cmap, const int32_t *prp, int32_t *pci, double *pv, hipStream_t s);
// The paper's classical, extended+i and hybrid interpolations
// (variant = CAMG_INTERP_*): per-row bound of the candidate list (returns
// the largest), set sizes (cnt) and the rows of P.  flags[0]: candidate
// list overflow; flags[1]: count and fill passes disagree.
// (xi_bounds also gives the largest bound of the rows not handled one thread
// per row; that one is passed to xi_count / xi_fill)
int xi_bounds(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int variant, int32_t *bnd, int *bmax_wave,
              Pool &tmp, hipStream_t s);
void xi_count(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int variant, const int32_t *bnd, int bmax,
              int32_t *cnt, int32_t *flags, hipStream_t s);
void xi_fill(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int variant, const int32_t *bnd, int bmax,
             const int64_t *cmap, const int32_t *prp, int32_t *pci, double *pv, int32_t *flags, hipStream_t s);
// BAMG prolongation: orthonormal basis of the test space (in place; nt <= 8),
// packed rows (nt slots per row, counts in cnt; flags[2]: a row has too
// many candidates), packed rows -> P (P.rp set), the next level's test space
void bamg_orthonormalize(int n, int nt, double *V, Pool &tmp, hipStream_t s);
void bamg_rows(int n, const Csr &A, const uint8_t *strong, const int8_t *cf, int nt, const double *V, int lmin,
               int lmax, double eps, double mu, const int64_t *cmap, int32_t *cnt, int32_t *tci, double *tv,
               int32_t *flags, hipStream_t s);
void bamg_compact(int n, int nt, const int32_t *tci, const double *tv, const Csr &P, hipStream_t s);
void bamg_gather_tv(int n, int nt, const int8_t *cf, const int64_t *cmap, const double *V, double *Vc, hipStream_t s);
// SRQM refinement of the orthonormal test space V (n x nt, in place) with
// M^{-1} = D^{-1} (G null) or G^T G; at most iters steps
void srqm(const Csr &A, const double *dinv, const Csr *G, const Csr *Gt, int nt, double *V, int iters, Pool &tmp,
          hipStream_t s);
// Prolongation smoothing P <- P - omega D^{-1} (A P), and filtering of P
// with compensation on the coarse test space W (n_c x nt); the new P is
// allocated from `out`.
void psmooth(const Csr &A, const double *dinv, double omega, Csr &P, Pool &out, Pool &tmp, hipStream_t s);
void pfilter(Csr &P, double rho, int nt, const double *W, Pool &out, Pool &tmp, hipStream_t s);
void fill_ones(int n, double *x, hipStream_t s);
void transpose_csr(const Csr &X, Csr &XT, Pool &tmp, hipStream_t s);
// FSAI smoother: counts of entries on or below the diagonal per row (returns
// the largest), the factor's rows (G.rp set, G.ci / G.v filled; flags[6]:
// row too long, flags[7]: not SPD), the power-method estimate of rho(G A G^T)
// rows of the FSAI factor: at most this many entries on or below the diagonal
constexpr int kFsaiMaxRow = 192;
int fsai_counts(int n, const int32_t *rp, const int32_t *ci, int32_t *cnt, Pool &tmp, hipStream_t s);
void fsai_rows(const Csr &A, Csr &G, int mmax, int32_t *flags, hipStream_t s);
// adaptive FSAI: rows padded to steps * step + 1 slots (pci / pv, counts in
// cnt; flags[6]: a candidate set exceeded 2048 entries, the level takes
// Jacobi; flags[7]: not SPD; flags[4]: internal capacity error), then
// compacted into G (G.rp the scan of the counts); tpos: transpose positions of A
void afsai_rows(const Csr &A, const int32_t *tpos, int maxrow, int steps, int step, double eps, int32_t *cnt,
                int32_t *pci, double *pv, int32_t *flags, hipStream_t s);
void afsai_compact(const Csr &G, int mcap, const int32_t *pci, const double *pv, hipStream_t s);
double fsai_rayleigh(const Csr &A, const Csr &G, const Csr &Gt, uint64_t seed, int level, Pool &tmp,
                     hipStream_t s);  // rho estimate of G A G^T for the FSAI weight
void column_counts(const Csr &X, int32_t *cnt, hipStream_t s);
void diag_gershgorin(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v, double *dinv,
                     unsigned long long *qmax_bits, int32_t *flags, hipStream_t s);
void scale_vec(int n, double omega, const double *dinv, double *wd, hipStream_t s);
void scale_columns(const Csr &A, const double *wd, double *awd, hipStream_t s);
void to_f32(int64_t n, const double *in, float *out, hipStream_t s);
void dense_from_csr(int n, const int32_t *rp, const int32_t *ci, const double *v, double *D, hipStream_t s);
void cholesky_dense(int n, double *D, int32_t *flags, hipStream_t s);
void chol_inverse(int n, const double *L, double *X, hipStream_t s);
int max_row_length(int n, const int32_t *rp, Pool &tmp, hipStream_t s);
// the same without a synchronisation: the longest row is folded into *out
// (zeroed by the caller)
void max_row_length_async(int n, const int32_t *rp, int32_t *out, hipStream_t s);
void tile_starts(int n, const int32_t *rp, int W, int ntiles, int32_t *tstart, hipStream_t s);
// compact columns: tile_bases_async places up to kTileWins windows of
// 2^kWinBits columns per tile (tbase: ntiles * kTileWins, slot 0 = the
// tile's smallest column) and leaves in flag[0..1] (zeroed by the caller)
// what the host turns into the mode: flag[1] == 0, one 65536-column span
// covers every tile (mode 1); else flag[0] == 0, the windows do (mode 2);
// else neither (0); tile_diffs then writes the 16-bit words of that mode
constexpr int kTileWins = 8, kWinBits = 13;
void tile_bases_async(int ntiles, const int32_t *tstart, const int32_t *rp, const int32_t *ci, int32_t *tbase,
                      int32_t *flag, hipStream_t s);
void tile_diffs(int ntiles, const int32_t *tstart, const int32_t *rp, const int32_t *ci, const int32_t *tbase,
                uint16_t *off, int mode, hipStream_t s);

// ---------------------------------------------------------------- SpGEMM (spgemm.hip)
// Z = X Y with the full symbolic pattern, rows sorted; for every output
// entry the products are added in ascending order of the inner index.
// Z's arrays are allocated from `out`.
void spgemm(const Csr &X, const Csr &Y, Csr &Z, Pool &out, Pool &tmp, hipStream_t s);
// A_c = R (A P); A P is formed in windows of at most `chunk` products
// (0: 2^30) when it would be larger; bitwise the same either way.
void galerkin(const Csr &A, const Csr &P, const Csr &R, Csr &Ac, int64_t chunk, Pool &out, Pool &tmp,
              hipStream_t s);

// ---------------------------------------------------------------- solve (solve.hip)
// the next row-kernel launch of the calling host thread records `start` and
// `stop` at the beginning and end of its execution (hipExtLaunchKernelGGL)
void time_next_row_launch(hipEvent_t start, hipEvent_t stop);
// drops a request no launch has taken yet; true if there was one
bool cancel_row_launch_timing();
RowCfg choose_cfg(int n, int64_t nnz, int maxrow);

// V-cycle building blocks.  T: value type of the level (double, or float
// in mixed precision); TY: type of the right-hand side y (level 0 reads
// the FP64 PCG residual); TZ: type of the output; DOT: write per-block
// partials of y.z (level 0 inside PCG).  st may be null (standalone
// V-cycle); otherwise the kernels return at once when st->done is set.
// awd (may be null): A's values scaled by wd of their column, so the first
// Jacobi step s_j = wd_j y_j needs one gather per nonzero instead of two.
template <class T, class TY>
void vc_pre(const Csr &A, const RowCfg &c, const T *wd, const T *awd, const TY *y, T *s, T *r, const PcgState *st,
            hipStream_t str);
template <class T, class TY, class TZ, bool DOT>
void vc_post(const Csr &A, const RowCfg &c, const T *wd, const TY *y, const T *s, TZ *z, double *partials,
             int32_t *nout, const PcgState *st, hipStream_t str);
template <class T, class TY>
void vc_resid(const Csr &A, const RowCfg &c, const TY *y, const T *s, T *r, const PcgState *st, hipStream_t str);
template <class T>
void vc_restrict(const Csr &R, const RowCfg &c, const T *r, T *yc, const PcgState *st, hipStream_t str);
template <class T>
void vc_prolong(const Csr &P, const RowCfg &c, const T *d, T *s, const PcgState *st, hipStream_t str);
// FSAI smoothing (M^{-1} = G^T G): u = G y; s = omega G^T u; z = s + omega G^T u
// (z may be s; with DOT the partials of y.z)
template <class T, class TY>
void vc_gmul(const Csr &G, const RowCfg &c, const TY *y, T *u, const PcgState *st, hipStream_t str);
template <class T>
void vc_fsai_first(const Csr &Gt, const RowCfg &c, T omega, const T *u, T *s, const PcgState *st, hipStream_t str);
template <class T, class TY, class TZ, bool DOT>
void vc_fsai_step(const Csr &Gt, const RowCfg &c, T omega, const T *u, const T *s, const TY *y, TZ *z,
                  double *partials, int32_t *nout, const PcgState *st, hipStream_t str);
template <class T>
void coarse_solve(int n, const double *cinv, const T *y, T *z, const PcgState *st, hipStream_t str);
// partial sums of y.z; returns the number of partials
int dot_partials(int n, const double *y, const double *z, double *partials, int32_t *nout, const PcgState *st,
                 hipStream_t s);

// PCG.  Each producer returns how many per-block partials it wrote.
int pcg_init(int n, const double *b, double *x, double *r, double *p0, double rtol, double *pr2, PcgState *st,
             hipStream_t s);
void pcg_check(const double *pr2, PcgState *st, double *hist, int hist_cap, int32_t *hflag, hipStream_t s);
int pcg_dir(const Csr &A, const RowCfg &c, const double *z, const double *pold, double *pnew, double *q,
            const double *prz, double *ppq, PcgState *st, hipStream_t s);
int pcg_update(int n, const double *p, const double *q, double *x, double *r, const double *ppq, double *pr2,
               PcgState *st, int32_t *hflag, hipStream_t s);
void pcg_restart(PcgState *st, hipStream_t s);
// partials of ||b - A x||^2 (and out = b - A x when out != null)
int residual_norm(const Csr &A, const RowCfg &c, const double *b, const double *x, double *out, double *partials,
                  int32_t *nout, hipStream_t s);
void sum_to(const double *partials, int n, double *out, hipStream_t s);

// ---------------------------------------------------------------- multi-RHS engine (multi.hip)
struct Engine;
// slot -> column of a right-hand-side block (-1: not involved); passed by value
struct SlotMap {
    int8_t q[kMaxSlots];
};
// per-column state copied out for the host (plain layout)
struct EngineSnap {
    int32_t iter[kMaxSlots], done[kMaxSlots], status[kMaxSlots], active[kMaxSlots];
    double rnorm[kMaxSlots], bnorm[kMaxSlots], tres2[kMaxSlots];
};
int64_t engine_footprint(const Hier &h, int K);
Engine *engine_create(Hier &h, int K, int cap, hipStream_t s);
void engine_destroy(Engine *e);
int engine_slots(const Engine &E);
// start columns [c0, c0+m) from the n-by-m row-major device block B (row stride ldb)
void engine_start(Engine &E, int c0, int m, const double *B, int ldb, double rtol, int max_iter, hipStream_t s);
// up to `iters` iterations; returns the number of columns still running
int engine_step(Engine &E, int iters, hipStream_t s);
void engine_slot_state(Engine &E, int32_t *iters, int32_t *done, int32_t *status, hipStream_t s);
void engine_true_res(Engine &E, double *rel, hipStream_t s);
void engine_copy_x(Engine &E, int c0, int m, double *X, int ldx, hipStream_t s);
void engine_release(Engine &E, int c0, int m, hipStream_t s);
void engine_replace(Engine &E, unsigned long long mask, hipStream_t s);
void engine_hist(Engine &E, int c, double *host, int cap_out, int count, hipStream_t s);
void engine_start_slots(Engine &E, const SlotMap &q, const double *B, int ldb, double rtol, int max_iter,
                        hipStream_t s);
void engine_launch(Engine &E, int iters, hipStream_t s);
void engine_snapshot(Engine &E, bool true_res, EngineSnap *snap, hipStream_t s);
void engine_release_mask(Engine &E, unsigned long long mask, hipStream_t s);
void engine_gather_x(Engine &E, const SlotMap &q, int k, double *out, hipStream_t s);
int engine_n(const Engine &E);

// ---------------------------------------------------------------- many small systems (batch.hip)
void solve_batch(std::vector<Hier *> &hs, const double *const *b, double *const *x, double rtol, int32_t *iters,
                 double *true_relres, int32_t *status, hipStream_t s, bool no_alloc);

// ---------------------------------------------------------------- server (serve.hip)
struct Server;
Server *server_create(int64_t budget);
int server_add(Server &S, Hier &h, int slots, int ipb);
void server_submit(Server &S, int sys, int k, const double *B, int ldb, double *X, int ldx, double rtol,
                   int max_iter, int64_t tag);
int server_poll(Server &S);
int server_take(Server &S, camg_completion *out, int cap);
void server_stats(const Server &S, int64_t *arena_used, int64_t *arena_size, int32_t *queued, int32_t *active);
void server_destroy(Server *S);

}  // namespace camg
