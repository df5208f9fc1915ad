// Many small systems at once: one persistent workgroup per system runs that
// system's whole PCG solve (every iteration, every V-cycle level, the
// last-level product, the stopping test and the true residual) inside a
// single kernel launch, with workgroup barriers as the only
// synchronisation.  Systems of different sizes and hierarchies share the
// launch; each workgroup reads its system's descriptor (device pointers of
// the handle's levels and work vectors).
//
// The arithmetic is the V-cycle of the single-vector path (pre-smoothing
// with the pre-scaled values a_ij w_j, restriction, last-level dense
// product, prolongation, post-smoothing) and the same PCG recurrence; rows
// are handled by groups of g lanes (g per matrix, from its mean row length)
// whose partial sums are combined by a fixed shuffle tree, and every dot
// product is a fixed-order workgroup reduction, so results are
// deterministic.  Meant for systems up to ~1e5 unknowns: one compute unit
// works through each system.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "devutil.hpp"
#include "internal.hpp"

namespace camg {
namespace {

constexpr int kBT = 1024;  // threads of a system's workgroup

template <class T>
struct BLev {
    int n = 0, nc = 0;         // rows of A_l, of A_{l+1}
    int ga = 1, gp = 1, gr = 1;  // lanes per row of A_l, P_l, R_l
    const int32_t *arp = nullptr, *aci = nullptr;
    const T *av = nullptr, *awd = nullptr, *wd = nullptr;
    const int32_t *prp = nullptr, *pci = nullptr;
    const T *pv = nullptr;
    const int32_t *rrp = nullptr, *rci = nullptr;
    const T *rv = nullptr;
    T *y = nullptr, *s = nullptr, *r = nullptr, *z = nullptr;  // level 0: s, r only
};

// the FP64 outer solver's part of a system (the same whatever the V-cycle precision)
struct BPcg {
    int nlev = 0, n = 0, nL = 0, max_iter = 0, mixed = 0;
    double rtol = 0.0;
    const double *cinv = nullptr;
    const double *b = nullptr;
    double *x = nullptr;
    const int32_t *arp = nullptr, *aci = nullptr;  // FP64 A_0 for q = A p and the true residual
    const double *av = nullptr;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
};

template <class T>
struct BSys : BPcg {
    BLev<T> lev[CAMG_MAX_LEVELS];
};

struct BOut {
    int32_t iters, status;
    double true_rel;
};

// sum over the workgroup in a fixed order; every thread gets the result
__device__ double wg_sum(double v) {
    __shared__ double ws[kBT / kWave];
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kBT / kWave; ++i) t += ws[i];
    __syncthreads();
    return t;
}

// group of g lanes (a power of two <= 64) per row: the lanes add the row's
// products in strides of g, then a shuffle tree combines them
template <class A, class X>
__device__ __forceinline__ A row_sum(const int32_t *rp, const int32_t *ci, const A *v, int i, int g, int lane, X x) {
    A acc = 0;
    const int e1 = rp[i + 1];
    for (int e = rp[i] + lane; e < e1; e += g) acc += v[e] * x(ci[e]);
    for (int o = g / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, g);
    return acc;
}

// for every row i of an n-row matrix with g lanes per row: f(i, acc) on the group's first lane
template <class F>
__device__ __forceinline__ void for_rows(int n, int g, F f) {
    const int lane = threadIdx.x & (g - 1);
    const int per = kBT / g;
    // every lane of a wavefront runs the same number of rounds so the
    // group shuffles always see their partners
    const int rounds = (n + per - 1) / per;
    for (int k = 0; k < rounds; ++k) {
        const int i = k * per + threadIdx.x / g;
        f(i < n ? i : -1, lane);
    }
}

template <class T>
__device__ void b_vcycle(const BSys<T> &S) {
    const int L = S.nlev - 1;
    // level 0 right-hand side is the PCG residual (FP64), its result the PCG z
    for (int l = 0; l < L; ++l) {
        const BLev<T> &V = S.lev[l];
        const double *y0 = S.r;
        // pre-smoothing: s = w y, r = y - (A w) y
        for_rows(V.n, V.ga, [&](int i, int lane) {
            T acc = 0;
            if (i >= 0) {
                if (l == 0) acc = row_sum<T>(V.arp, V.aci, V.awd, i, V.ga, lane, [&](int j) { return (T)y0[j]; });
                else acc = row_sum<T>(V.arp, V.aci, V.awd, i, V.ga, lane, [&](int j) { return V.y[j]; });
            } else {
                for (int o = V.ga / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, V.ga);
            }
            if (i >= 0 && lane == 0) {
                const T yi = l == 0 ? (T)y0[i] : V.y[i];
                V.s[i] = V.wd[i] * yi;
                V.r[i] = yi - acc;
            }
        });
        __syncthreads();
        // restriction: y_{l+1} = R r
        const BLev<T> &C = S.lev[l + 1];
        for_rows(V.nc, V.gr, [&](int i, int lane) {
            T acc = 0;
            if (i >= 0) acc = row_sum<T>(V.rrp, V.rci, V.rv, i, V.gr, lane, [&](int j) { return V.r[j]; });
            else
                for (int o = V.gr / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, V.gr);
            if (i >= 0 && lane == 0) C.y[i] = acc;
        });
        __syncthreads();
    }
    // last level: z = A_L^{-1} y (FP64 products)
    {
        const BLev<T> &V = S.lev[L];
        const int g = 64;
        for_rows(S.nL, g, [&](int i, int lane) {
            double acc = 0.0;
            if (i >= 0) {
                const double *row = S.cinv + (size_t)i * S.nL;
                if (L == 0)
                    for (int j = lane; j < S.nL; j += g) acc += row[j] * S.r[j];
                else
                    for (int j = lane; j < S.nL; j += g) acc += row[j] * (double)V.y[j];
            }
            acc = wave_sum(acc);
            if (i >= 0 && lane == 0) {
                if (L == 0) S.z[i] = acc;
                else V.z[i] = (T)acc;
            }
        });
        __syncthreads();
    }
    for (int l = L - 1; l >= 0; --l) {
        const BLev<T> &V = S.lev[l];
        const BLev<T> &C = S.lev[l + 1];
        // prolongation and correction: s += P z_{l+1}
        for_rows(V.n, V.gp, [&](int i, int lane) {
            T acc = 0;
            if (i >= 0) acc = row_sum<T>(V.prp, V.pci, V.pv, i, V.gp, lane, [&](int j) { return C.z[j]; });
            else
                for (int o = V.gp / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, V.gp);
            if (i >= 0 && lane == 0) V.s[i] = V.s[i] + acc;
        });
        __syncthreads();
        // post-smoothing: z = s + w (y - A s)
        for_rows(V.n, V.ga, [&](int i, int lane) {
            T acc = 0;
            if (i >= 0) acc = row_sum<T>(V.arp, V.aci, V.av, i, V.ga, lane, [&](int j) { return V.s[j]; });
            else
                for (int o = V.ga / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, V.ga);
            if (i >= 0 && lane == 0) {
                const T yi = l == 0 ? (T)S.r[i] : V.y[i];
                const T zi = V.s[i] + V.wd[i] * (yi - acc);
                if (l == 0) S.z[i] = (double)zi;
                else V.z[i] = zi;
            }
        });
        __syncthreads();
    }
}

// ||b - A x||^2 on the FP64 A_0; stores the residual into S.r when store
__device__ double b_true_res2(const BPcg &S, bool store) {
    double part = 0.0;
    const int g = 8;
    for_rows(S.n, g, [&](int i, int lane) {
        double acc = 0.0;
        if (i >= 0) acc = row_sum<double>(S.arp, S.aci, S.av, i, g, lane, [&](int j) { return S.x[j]; });
        else
            for (int o = g / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, g);
        if (i >= 0 && lane == 0) {
            const double d = S.b[i] - acc;
            if (store) S.r[i] = d;
            part += d * d;
        }
    });
    return wg_sum(part);
}

template <class T>
__global__ void __launch_bounds__(kBT) kb_solve(const BSys<T> *sys, BOut *out) {
    const BSys<T> &S = sys[blockIdx.x];
    const BPcg &D = S;
    const int n = S.n;
    double bb = 0.0;
    for (int i = threadIdx.x; i < n; i += kBT) {
        const double bi = S.b[i];
        S.x[i] = 0.0;
        S.r[i] = bi;
        S.p[i] = 0.0;
        bb += bi * bi;
    }
    const double bnorm = sqrt(wg_sum(bb));
    const double tol = S.rtol > 0.0 ? S.rtol * bnorm : -1.0;
    int it = 0, restart = 0, reps = 0, status = CAMG_OK;
    double rho_old = 0.0, rn2 = bnorm * bnorm;
    while (true) {
        const double rn = sqrt(rn2);
        if (bnorm == 0.0 || (tol > 0.0 && rn < tol)) {
            // mixed precision: the true residual must pass too (restart from it, at most twice)
            if (!S.mixed || bnorm == 0.0 || reps >= 2 || it >= S.max_iter) break;
            const double t2 = b_true_res2(D, false);
            if (sqrt(t2) < tol) break;
            rn2 = b_true_res2(D, true);
            restart = it;
            ++reps;
            __syncthreads();
            continue;
        }
        if (it >= S.max_iter) {
            status = CAMG_E_MAXIT;
            break;
        }
        b_vcycle<T>(S);
        double rz = 0.0;
        for (int i = threadIdx.x; i < n; i += kBT) rz += S.r[i] * S.z[i];
        const double rho = wg_sum(rz);
        const double beta = it == restart ? 0.0 : rho / rho_old;
        for (int i = threadIdx.x; i < n; i += kBT) S.p[i] = S.z[i] + beta * S.p[i];
        __syncthreads();
        double pq = 0.0;
        for_rows(n, 8, [&](int i, int lane) {
            double acc = 0.0;
            if (i >= 0) acc = row_sum<double>(S.arp, S.aci, S.av, i, 8, lane, [&](int j) { return S.p[j]; });
            else
                for (int o = 4; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 8);
            if (i >= 0 && lane == 0) {
                S.q[i] = acc;
                pq += S.p[i] * acc;
            }
        });
        const double sigma = wg_sum(pq);
        if (!(sigma > 0.0) || !(rho > 0.0)) {
            status = CAMG_E_BREAKDOWN;
            break;
        }
        const double alpha = rho / sigma;
        double r2 = 0.0;
        for (int i = threadIdx.x; i < n; i += kBT) {
            S.x[i] = S.x[i] + alpha * S.p[i];
            const double ri = S.r[i] - alpha * S.q[i];
            S.r[i] = ri;
            r2 += ri * ri;
        }
        rn2 = wg_sum(r2);
        rho_old = rho;
        ++it;
    }
    const double t2 = b_true_res2(D, false);
    // mixed precision: a recursive stop whose true residual still fails after
    // the restarts is an accuracy warning
    if (S.mixed && status == CAMG_OK && tol > 0.0 && !(sqrt(t2) < tol)) status = CAMG_E_ACCURACY;
    if (threadIdx.x == 0) {
        out[blockIdx.x].iters = it;
        out[blockIdx.x].status = status;
        out[blockIdx.x].true_rel = bnorm > 0.0 ? sqrt(t2) / bnorm : 0.0;
    }
}

int lanes_for(const Csr &M) {
    const double mean = M.nr > 0 ? (double)M.nnz / M.nr : 1.0;
    int g = 1;
    while (g < 32 && g < mean) g <<= 1;
    return g;
}

template <class T>
const T *vals(const Csr &M);
template <>
const double *vals<double>(const Csr &M) { return M.v; }
template <>
const float *vals<float>(const Csr &M) { return M.v32; }

template <class T>
BSys<T> describe(Hier &h, const double *b, double *x, double rtol) {
    BSys<T> S;
    S.nlev = h.nlev;
    S.n = h.lev[0].A.nr;
    S.nL = h.nL;
    S.max_iter = h.prm.max_iter;
    S.mixed = h.prm.precision == CAMG_MIXED_FP32;
    S.rtol = rtol;
    S.cinv = h.cinv;
    S.b = b;
    S.x = x;
    S.arp = h.lev[0].A.rp;
    S.aci = h.lev[0].A.ci;
    S.av = h.lev[0].A.v;
    S.r = h.r;
    S.z = h.z;
    S.p = h.p[0];
    S.q = h.q;
    for (int l = 0; l < h.nlev; ++l) {
        Level &L = h.lev[l];
        BLev<T> &V = S.lev[l];
        V.n = L.A.nr;
        V.ga = lanes_for(L.A);
        V.arp = L.A.rp;
        V.aci = L.A.ci;
        V.av = vals<T>(L.A);
        if constexpr (sizeof(T) == 8) {
            V.awd = L.awd;
            V.wd = L.wd;
            V.y = L.y;
            V.s = L.s;
            V.r = L.r;
            V.z = L.z;
        } else {
            V.awd = L.awd32;
            V.wd = L.wd32;
            V.y = L.y32;
            V.s = L.s32;
            V.r = L.r32;
            V.z = L.z32;
        }
        if (l < h.nlev - 1) {
            V.nc = L.P.nc;
            V.gp = lanes_for(L.P);
            V.gr = lanes_for(L.R);
            V.prp = L.P.rp;
            V.pci = L.P.ci;
            V.pv = vals<T>(L.P);
            V.rrp = L.R.rp;
            V.rci = L.R.ci;
            V.rv = vals<T>(L.R);
        }
    }
    return S;
}

// Descriptors in, results out, one launch: dsys holds m BSys<T>, dout m BOut
// (device memory of the caller's choosing, left as the launch wrote it).
template <class T>
void launch_batch(std::vector<Hier *> &hs, const double *const *b, double *const *x, double rtol, void *dsys,
                  void *dout, std::vector<BOut> &out, hipStream_t s) {
    const int m = (int)hs.size();
    std::vector<BSys<T>> host(m);
    for (int k = 0; k < m; ++k) host[k] = describe<T>(*hs[k], b[k], x[k], rtol);
    HIPC(hipMemcpyAsync(dsys, host.data(), sizeof(BSys<T>) * m, hipMemcpyHostToDevice, s));
    kb_solve<T><<<m, kBT, 0, s>>>(static_cast<const BSys<T> *>(dsys), static_cast<BOut *>(dout));
    HIPC(hipGetLastError());
    out.resize(m);
    HIPC(hipMemcpyAsync(out.data(), dout, sizeof(BOut) * m, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
}

template <class T>
void run_batch(std::vector<Hier *> &hs, const double *const *b, double *const *x, double rtol, std::vector<BOut> &out,
               hipStream_t s) {
    const int m = (int)hs.size();
    void *dsys = nullptr, *dout = nullptr;
    HIPC(hipMalloc(&dsys, sizeof(BSys<T>) * m));
    struct Free {
        void **a, **b;
        ~Free() {
            if (*a) (void)hipFree(*a);
            if (*b) (void)hipFree(*b);
        }
    } fr{&dsys, &dout};
    HIPC(hipMalloc(&dout, sizeof(BOut) * m));
    launch_batch<T>(hs, b, x, rtol, dsys, dout, out, s);
}

// ---- allocation-free variant: descriptors and results in a static device array
//
// Each GPU the library runs on holds one copy of `scratch` until the process
// ends.  Its device address is taken once per device (with that device
// current) and kept; host code never passes the array's own name to a
// kernel or a copy.  The descriptors start at offset 0, the results at
// kOutOff; a call overwrites every byte it reads back, so nothing has to
// start at zero.
constexpr size_t kDescBytes = sizeof(BSys<double>);
static_assert(sizeof(BSys<float>) == kDescBytes, "descriptor sizes of both precisions are equal");
constexpr size_t kOutOff = ((size_t)CAMG_NOALLOC_MAX_SYSTEMS * kDescBytes + 255) / 256 * 256;
constexpr size_t kScratchBytes = kOutOff + ((size_t)CAMG_NOALLOC_MAX_SYSTEMS * sizeof(BOut) + 255) / 256 * 256;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// the calling thread's current device must be dev
void *scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(CAMG_E_DEVICE, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) fail(CAMG_E_DEVICE, "hipGetSymbolAddress of the batch scratch array failed");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

// Solve count systems, one workgroup each, in one launch (handles of one
// precision, one smoothing step each way).  no_alloc: the descriptors and
// results live in the static scratch array of the current device instead of
// two allocations of this call.
void solve_batch(std::vector<Hier *> &hs, const double *const *b, double *const *x, double rtol, int32_t *iters,
                 double *true_relres, int32_t *status, hipStream_t s, bool no_alloc) {
    const int prec = hs[0]->prm.precision;
    for (Hier *h : hs) {
        if (h->prm.precision != prec) fail(CAMG_E_ARG, "all handles of a batch must have the same precision");
        if (h->prm.nu_pre != 1 || h->prm.nu_post != 1)
            fail(CAMG_E_ARG, "the batched solver runs one smoothing step each way");
        if (h->prm.smoother != CAMG_SMOOTH_JACOBI) fail(CAMG_E_ARG, "the batched solver runs the Jacobi smoother only");
        if (h->device != hs[0]->device) fail(CAMG_E_ARG, "all handles of a batch must live on one device");
    }
    std::vector<BOut> out;
    if (no_alloc) {
        if (hs.size() > (size_t)CAMG_NOALLOC_MAX_SYSTEMS)
            fail(CAMG_E_ARG, "more systems than the allocation-free batch holds (CAMG_NOALLOC_MAX_SYSTEMS)");
        int dev = -1;
        HIPC(hipGetDevice(&dev));
        unsigned char *base = static_cast<unsigned char *>(scratch_ptr(dev));
        if (prec == CAMG_MIXED_FP32) launch_batch<float>(hs, b, x, rtol, base, base + kOutOff, out, s);
        else launch_batch<double>(hs, b, x, rtol, base, base + kOutOff, out, s);
    } else if (prec == CAMG_MIXED_FP32) {
        run_batch<float>(hs, b, x, rtol, out, s);
    } else {
        run_batch<double>(hs, b, x, rtol, out, s);
    }
    for (size_t k = 0; k < hs.size(); ++k) {
        if (iters) iters[k] = out[k].iters;
        if (true_relres) true_relres[k] = out[k].true_rel;
        if (status) status[k] = out[k].status;
    }
}

}  // namespace camg
