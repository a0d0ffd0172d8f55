// Host side of the C ABI declared in include/lgf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lgf.h"
#include "fft.hpp"
#include "kernels.hpp"

using namespace lgf;

namespace {

thread_local std::string g_create_error;

constexpr int HIST_CAP = 1 << 16;
constexpr size_t ZT_LDS_BUDGET = 80 * 1024;  // bytes of LDS per (z,t) tile
constexpr int FP32_STALL_SWEEPS = 6;  // FP32 sweeps without a new theta minimum: hand over

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double seconds() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

}  // namespace

struct lgf_ctx {
    geom g{};
    int precision = LGF_FP64;
    int device = 0;
    hipStream_t stream = nullptr;
    double p2max = 0;
    double theta_switch = 1e-8;
    bool accelerate = true;  // false: plain steepest descent (no transform)
    bool exact_exp = false;  // true: g = exp((alpha/2) L Delta) exactly
    double half_alpha = 0;   // alpha/2 of the sweeps being enqueued (FP64 G accumulation)

    // working links (SoA; 12-real by default, 18-real or SU(2) row 0 by the
    // context's format): FP64 double buffer; the FP32 pair aliases L64[1]
    double2 *L64[2] = {nullptr, nullptr};
    float2 *L32[2] = {nullptr, nullptr};
    float2 *G32 = nullptr;
    // Fourier fields (4 complex per site), FP64 size; FP32 views alias them
    double2 *D64[2] = {nullptr, nullptr};
    // tables: per-axis twiddles (x, y, z, t tables one after the other) and
    // per-axis p2 by transform position
    double2 *tw64 = nullptr;
    float2 *tw32 = nullptr;
    double *pt64 = nullptr;
    float *pt32 = nullptr;
    fft_plan plan64{}, plan32{};  // how the transform is split into passes
    // reductions and control
    double *partials = nullptr;
    int nparts = 0;
    dev_status *status = nullptr;
    dev_status *status_host = nullptr;  // pinned, 3 slots: synchronous reads, two batches
    hipEvent_t batch_ev[2] = {nullptr, nullptr};  // a batch's status copy has landed
    double *reduce_out = nullptr;       // device [2]
    double *reduce_host = nullptr;      // pinned [2]
    double *histF = nullptr, *histT = nullptr;
    int hist_len = 0;
    // differentiation scratch (allocated on first use)
    double *gaos = nullptr;   // V*9 complex or 4V*9 complex (link exponentials)
    double2 *Lrot = nullptr;  // 12-real FP64 links (differentiation scratch)
    // exactly exponentiated g, rows 0,1 (SU(3) exact step; allocated when enabled)
    double2 *Gex = nullptr;
    std::string err;
};

namespace {

int fail(lgf_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, LGF_ERR_DEVICE,                                                  \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    } while (0)

// F = normF sum Re Tr U, theta = normT sum Tr[Delta Delta^+] (Nd = 4, Nc = g.nc)
double normF(const lgf_ctx *c) { return 1.0 / (4.0 * c->g.nc * (double)c->g.V); }
double normT(const lgf_ctx *c) { return 1.0 / ((double)c->g.nc * (double)c->g.V); }

// Stopping-test parameters for the sweep kernels (enabled == false: the
// kernel only writes block partials).
fin_params finp(const lgf_ctx *c, bool enabled, double tol = 0, int max_iter = 0,
                int increment = 0, int stall = 0) {
    fin_params f;
    f.stall = stall;
    f.normF = normF(c);
    f.normT = normT(c);
    f.tol = tol;
    f.max_iter = max_iter;
    f.increment = increment;
    f.hist_cap = HIST_CAP;
    f.enabled = enabled ? 1 : 0;
    f.histF = c->histF;
    f.histT = c->histT;
    return f;
}

// The axis tables exp(-2 pi i j / L_mu), j < L_mu, of x, y, z and t one after
// the other, from long double.
template <class V2> std::vector<V2> make_twiddles(const geom &g) {
    const int L[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
    std::vector<V2> t;
    const long double twopi = 6.283185307179586476925286766559005768L;
    for (int mu = 0; mu < 4; ++mu)
        for (int j = 0; j < L[mu]; ++j) {
            const long double a = twopi * (long double)j / (long double)L[mu];
            V2 v;
            v.x = (decltype(v.x))cosl(a);
            v.y = (decltype(v.y))(-sinl(a));
            t.push_back(v);
        }
    return t;
}

// Per-axis 4 sin^2(pi k / L) indexed by transform position (see fft_freq_of_pos).
std::vector<long double> make_p2_tables(const geom &g, long double &p2max) {
    const int L[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> t;
    p2max = 0;
    for (int mu = 0; mu < 4; ++mu) {
        long double mx = 0;
        for (int p = 0; p < L[mu]; ++p) {
            const int k = fft_freq_of_pos(L[mu], p);
            const long double s = sinl(pi * (long double)k / (long double)L[mu]);
            t.push_back(4.0L * s * s);
            if (4.0L * s * s > mx) mx = 4.0L * s * s;
        }
        p2max += mx;
    }
    return t;
}

// Every extent 2^a 3^b in [2, FFT_MAX_EXTENT]; the volume below 2^31 sites
// (site coordinates are decoded in 32-bit arithmetic).
bool shape_ok(const int L[4]) {
    long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (!fft_supported(L[mu])) return false;
        V *= L[mu];
    }
    return V < (1L << 31);
}

// ------------------------------------------------------------------ sweep

template <class T> struct prec;
template <> struct prec<double> {
    static void *links(lgf_ctx *c, int i) { return c->L64[i]; }
    static void *field(lgf_ctx *c, int i) { return c->D64[i]; }
    static const void *tw(lgf_ctx *c) { return c->tw64; }
    static const double *pt(lgf_ctx *c) { return c->pt64; }
    static const fft_plan &W(lgf_ctx *c) { return c->plan64; }
};
template <> struct prec<float> {
    static void *links(lgf_ctx *c, int i) { return c->L32[i]; }
    static void *field(lgf_ctx *c, int i) { return c->D64[i]; }
    static const void *tw(lgf_ctx *c) { return c->tw32; }
    static const float *pt(lgf_ctx *c) { return c->pt32; }
    static const fft_plan &W(lgf_ctx *c) { return c->plan32; }
};

// The accumulated transformation of the FP32 sweeps after n of them.  SU(3)
// alternates between G32 and the second FP32 link buffer (free there: the
// FP32 sweeps keep the constant copy U0 in L32[0] and form G U0 G^dagger);
// SU(2) updates G32 in place.
float2 *acc_G(lgf_ctx *c, int n) { return (c->g.nc == 3 && (n & 1)) ? c->L32[1] : c->G32; }

// Arguments of launch_update for the sweep from buffer `cur` into `cur^1`.
template <class T>
hipError_t sweep_update(lgf_ctx *c, int cur, void *D, T half_alpha, const fin_params &fp) {
    using P = prec<T>;
    if constexpr (std::is_same<T, float>::value) {
        if (c->g.nc == 3)
            return launch_update<T>(c->g, c->L32[0], nullptr, D, P::field(c, cur ^ 1),
                                    acc_G(c, cur), half_alpha, c->exact_exp, acc_G(c, cur ^ 1),
                                    c->partials, c->status, fp, c->stream);
    }
    return launch_update<T>(c->g, P::links(c, cur), P::links(c, cur ^ 1), D, P::field(c, cur ^ 1),
                            std::is_same<T, float>::value ? c->G32 : nullptr, half_alpha,
                            c->exact_exp, c->Gex, c->partials, c->status, fp, c->stream);
}

// One of the three transform passes of a sweep on the Fourier field D (0: (x,y)
// forward, 1: (z,t) forward / scaling / inverse, 2: (x,y) inverse), in the
// field's precision: FP32 for FP32 sweeps and for FP64 sweeps with g.ff32.
template <class T> bool field32(const lgf_ctx *c) {
    return std::is_same<T, float>::value || c->g.ff32;
}
hipError_t transform_pass(lgf_ctx *c, bool f32, int pass, void *D) {
    const double k = c->p2max / (double)c->g.V;
    if (f32) {
        if (pass == 0)
            return launch_fft_xy<float>(c->g, D, -1, c->tw32, c->plan32, c->status, c->stream);
        if (pass == 1)
            return launch_fft_zt<float>(c->g, D, 0, c->tw32, c->pt32, (float)k, c->plan32,
                                        c->status, c->stream);
        return launch_fft_xy<float>(c->g, D, +1, c->tw32, c->plan32, c->status, c->stream);
    }
    if (pass == 0)
        return launch_fft_xy<double>(c->g, D, -1, c->tw64, c->plan64, c->status, c->stream);
    if (pass == 1)
        return launch_fft_zt<double>(c->g, D, 0, c->tw64, c->pt64, k, c->plan64, c->status,
                                     c->stream);
    return launch_fft_xy<double>(c->g, D, +1, c->tw64, c->plan64, c->status, c->stream);
}

// Pass `pass` (0..2) of sweep `cur`'s transform of field D (none without the
// acceleration).  In the FP32 sweeps of an SU(3) mixed solve pass 2 also
// accumulates G <- g G: fused into the inverse (x,y) pass when one block can
// hold a plane of all four fields (xy_acc_fusable), else as a kernel after it.
template <class T>
hipError_t sweep_pass(lgf_ctx *c, int cur, void *D, T half_alpha, int pass) {
    if constexpr (std::is_same<T, float>::value) {
        if (c->g.nc == 3 && pass == 2) {
            if (c->accelerate && xy_acc_fusable<float>(c->g, c->plan32))
                return launch_fft_xy_inv_acc<float>(c->g, D, c->tw32, c->plan32, acc_G(c, cur),
                                                    acc_G(c, cur ^ 1), c->half_alpha, c->exact_exp,
                                                    c->status, c->stream);
            if (c->accelerate) {
                const hipError_t e = transform_pass(c, true, 2, D);
                if (e != hipSuccess) return e;
            }
            return launch_gauge_acc(c->g, D, acc_G(c, cur), acc_G(c, cur ^ 1), c->half_alpha,
                                    c->exact_exp, c->status, c->stream);
        }
    }
    if (!c->accelerate) return hipSuccess;
    return transform_pass(c, field32<T>(c), pass, D);
}

// One Fourier-accelerated sweep from links/field buffer `cur` into `cur^1`.
template <class T>
hipError_t enqueue_sweep(lgf_ctx *c, int cur, T half_alpha, const fin_params &fp) {
    using P = prec<T>;
    hipError_t e;
    void *D = P::field(c, cur);
    for (int pass = 0; pass < 3; ++pass)
        if ((e = sweep_pass<T>(c, cur, D, half_alpha, pass)) != hipSuccess) return e;
    return sweep_update<T>(c, cur, D, half_alpha, fp);
}

int read_status(lgf_ctx *c, dev_status &out) {
    HIPCHK(c, hipMemcpyAsync(c->status_host, c->status, sizeof(dev_status), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out = *c->status_host;
    return LGF_OK;
}

// Runs one precision phase on the working links in buffer 0.  On return the
// current links (FP64) or accumulated transformation (FP32, acc_G) are those
// after n = st.n sweeps and `st` holds the final state.
// prepared: the status reset and the first divergence with its stopping test
// were enqueued by the caller (the mixed hand-over fuses them).
//
// Sweeps go to the stream in batches.  After each batch the device status is
// copied to a pinned host slot (two slots, alternating, each with an event),
// and the next batch is enqueued before the host waits for the previous
// one's status, so the device does not idle while the host decides: a solve
// sizes each batch from the contraction rate last observed, counting the
// sweeps still in flight; once the stopping test has fired, sweeps still in
// flight find the device flag set and return at once.  A fixed count of
// sweeps (tol <= 0) goes in batches of 64.
template <class T>
int run_phase(lgf_ctx *c, double alpha, double tol, int max_iter, int hist_base, dev_status &st,
              int stall = 0, bool prepared = false) {
    if (!prepared) {
        HIPCHK(c, launch_status_reset(c->status, hist_base, c->stream));
        HIPCHK(c, launch_div_reduce<T>(c->g, prec<T>::links(c, 0), prec<T>::field(c, 0),
                                       c->partials, c->status,
                                       finp(c, true, tol, max_iter, 0, stall), c->stream));
    }
    int rc = read_status(c, st);
    if (rc) return rc;
    const T half_alpha = (T)(0.5 * alpha);
    c->half_alpha = 0.5 * alpha;
    const fin_params fp = finp(c, true, tol, max_iter, 1, stall);
    int enq = 0;              // sweeps enqueued so far
    double th_prev = st.theta;  // the observation before the last one (rate)
    int n_prev = st.n;
    // sweeps to enqueue next, from the last observed state and the sweeps
    // enqueued beyond it.  A solve caps its batches at max(4, n/8): the
    // contraction rate of the accelerated method rises several-fold in its
    // last decades, so a prediction from the rate so far overshoots, and every
    // sweep enqueued past the stop still costs its (empty) launches; with two
    // batches in flight, small batches cost no idle time.
    auto next_batch = [&]() {
        int k = tol > 0 ? 4 : 64;
        if (tol > 0 && st.n > n_prev && st.theta > 0 && th_prev > 0) {
            double rate = std::pow(st.theta / th_prev, 1.0 / (double)(st.n - n_prev));
            rate = std::min(std::max(rate, 1e-3), 0.95);
            const double need = std::log(tol / st.theta) / std::log(rate) - (double)(enq - st.n);
            k = (int)std::ceil(std::min(std::max(need, 1.0), 64.0));
            k = std::min(k, std::max(4, st.n / 8));
        }
        k = std::max(1, std::min(k, 64));
        return std::min(k, max_iter - enq);
    };
    auto enqueue_batch = [&](int k, int slot) -> int {
        for (int i = 0; i < k; ++i) {
            const int cur = (enq + i) & 1;
            HIPCHK(c, enqueue_sweep<T>(c, cur, half_alpha, fp));
        }
        enq += k;
        HIPCHK(c, hipMemcpyAsync(c->status_host + 1 + slot, c->status, sizeof(dev_status),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipEventRecord(c->batch_ev[slot], c->stream));
        return LGF_OK;
    };
    int queued = 0, observed = 0;  // batches enqueued / whose status was read
    while (!st.done) {
        // keep two batches in flight: enqueue the next one (at least one
        // sweep, so the device is never idle before the stop) unless every
        // allowed sweep is already enqueued
        if (queued - observed < 2) {
            const int k = next_batch();
            if (k > 0) {
                if ((rc = enqueue_batch(k, queued & 1))) return rc;
                ++queued;
                continue;
            }
        }
        if (observed == queued) {
            // nothing in flight and no sweep left to enqueue: the last
            // sweep's test must have ended the phase; read it
            rc = read_status(c, st);
            if (rc) return rc;
            if (!st.done) return fail(c, LGF_ERR_DEVICE, "sweep count exhausted without a stop");
            break;
        }
        HIPCHK(c, hipEventSynchronize(c->batch_ev[observed & 1]));
        th_prev = st.theta;
        n_prev = st.n;
        st = c->status_host[1 + (observed & 1)];
        ++observed;
    }
    // sweeps enqueued after the stop return at once; let them drain
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGF_OK;
}

int status_to_code(int code) {
    switch (code) {
    case ST_CONVERGED: return LGF_OK;
    case ST_MAXITER: return LGF_NOT_CONVERGED;
    case ST_NONFINITE: return LGF_ERR_NONFINITE;
    case ST_DIVERGING: return LGF_DIVERGING;
    case ST_STALLED: return LGF_NOT_CONVERGED;
    default: return LGF_OK;
    }
}

// Geometry for the entry points that always work on 12-real links (they pack
// the caller's links themselves).
geom g12(const lgf_ctx *c) {
    geom g = c->g;
    g.lf = 12;
    g.ff32 = 0;  // these entry points read the field back in FP64
    return g;
}

// (Re)allocate the working link buffers for the context's link format: each
// holds 4 links x (lf/2 for SU(3), 2 for SU(2)) complex entries per site
// (FP64), and never fewer than the 12-real form needs, because the per-step
// entry points pack 12-real links into buffer 0 whatever the format; the
// FP32 pair aliases the second buffer.
bool alloc_links(lgf_ctx *c) {
    for (auto &p : c->L64) {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    const size_t n = (size_t)4 * (c->g.nc == 2 ? 2 : std::max(c->g.lf, 12) / 2) * c->g.S;
    for (auto &p : c->L64)
        if (hipMalloc((void **)&p, n * sizeof(double2)) != hipSuccess) return false;
    c->L32[0] = reinterpret_cast<float2 *>(c->L64[1]);
    c->L32[1] = reinterpret_cast<float2 *>(c->L64[1]) + n;
    return true;
}

int check_ctx(lgf_ctx *c) {
    if (!c) return LGF_ERR_ARG;
    if (!c->L64[0] || !c->L64[1])
        return fail(c, LGF_ERR_OOM, "link buffers lost in a failed format change");
    HIPCHK(c, hipSetDevice(c->device));
    return LGF_OK;
}

// Pack caller links into FP64 working buffer 0 (12-real form), then F/theta
// of them.
int eval_links64(lgf_ctx *c, const double *U, double &F, double &theta) {
    const geom g = g12(c);
    HIPCHK(c, launch_pack_links<double>(U, c->L64[0], g, c->stream));
    HIPCHK(c, launch_status_reset(c->status, 0, c->stream));
    HIPCHK(c, launch_div_reduce<double>(g, c->L64[0], c->D64[0], c->partials, c->status,
                                        finp(c, false), c->stream));
    HIPCHK(c, launch_reduce_only(c->partials, c->nparts, c->reduce_out, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->reduce_host, c->reduce_out, 2 * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    F = c->reduce_host[0] * normF(c);
    theta = c->reduce_host[1] * normT(c);
    return LGF_OK;
}

int ensure_diff_scratch(lgf_ctx *c) {
    if (!c->gaos) {
        if (hipMalloc(&c->gaos, (size_t)4 * c->g.V * 9 * sizeof(double2)) != hipSuccess)
            return fail(c, LGF_ERR_OOM, "out of device memory (differentiation scratch)");
    }
    if (!c->Lrot) {
        if (hipMalloc(&c->Lrot, (size_t)24 * c->g.S * sizeof(double2)) != hipSuccess)
            return fail(c, LGF_ERR_OOM, "out of device memory (differentiation scratch)");
    }
    return LGF_OK;
}

int sum_partials(lgf_ctx *c, double &A, double &B) {
    HIPCHK(c, launch_reduce_only(c->partials, c->nparts, c->reduce_out, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->reduce_host, c->reduce_out, 2 * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    A = c->reduce_host[0];
    B = c->reduce_host[1];
    return LGF_OK;
}

template <class T>
int profile_impl(lgf_ctx *c, const double *U, double alpha, int n, double *ms) {
    using P = prec<T>;
    const bool accG = std::is_same<T, float>::value;
    HIPCHK(c, launch_pack_links<T>(U, P::links(c, 0), c->g, c->stream));
    if (accG) HIPCHK(c, launch_g_identity(c->G32, c->g, c->stream));
    HIPCHK(c, launch_status_reset(c->status, 0, c->stream));
    HIPCHK(c, launch_div_reduce<T>(c->g, P::links(c, 0), P::field(c, 0), c->partials, c->status,
                                   finp(c, true, 0.0, n + 1, 0), c->stream));
    std::vector<hipEvent_t> ev((size_t)n * 6);
    for (auto &e : ev) HIPCHK(c, hipEventCreate(&e));
    const T half_alpha = (T)(0.5 * alpha);
    c->half_alpha = 0.5 * alpha;
    int rc = LGF_OK;
    for (int it = 0; it < n && rc == LGF_OK; ++it) {
        const int cur = it & 1;
        void *D = P::field(c, cur);
        hipEvent_t *e = &ev[(size_t)it * 6];
        hipError_t err = hipSuccess;
        auto chk = [&](hipError_t x) { if (err == hipSuccess) err = x; };
        chk(hipEventRecord(e[0], c->stream));
        chk(sweep_pass<T>(c, cur, D, half_alpha, 0));
        chk(hipEventRecord(e[1], c->stream));
        chk(sweep_pass<T>(c, cur, D, half_alpha, 1));
        chk(hipEventRecord(e[2], c->stream));
        chk(sweep_pass<T>(c, cur, D, half_alpha, 2));
        chk(hipEventRecord(e[3], c->stream));
        chk(sweep_update<T>(c, cur, D, half_alpha, finp(c, false)));
        chk(hipEventRecord(e[4], c->stream));
        chk(launch_finalize(c->partials, c->nparts, c->status, finp(c, true, 0.0, n + 1, 1),
                            c->stream));
        chk(hipEventRecord(e[5], c->stream));
        if (err != hipSuccess) rc = fail(c, LGF_ERR_DEVICE, hipGetErrorString(err));
    }
    if (rc == LGF_OK) {
        hipError_t err = hipStreamSynchronize(c->stream);
        for (int k = 0; k < 5; ++k) ms[k] = 0;
        for (int it = 0; it < n && err == hipSuccess; ++it)
            for (int k = 0; k < 5 && err == hipSuccess; ++k) {
                float t = 0;
                err = hipEventElapsedTime(&t, ev[(size_t)it * 6 + k], ev[(size_t)it * 6 + k + 1]);
                ms[k] += t / n;
            }
        if (err != hipSuccess) rc = fail(c, LGF_ERR_DEVICE, hipGetErrorString(err));
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return rc;
}

// ------------------------------------------------- fixed scratch (no allocation)

// Block partial sums of lgf_measure_noalloc: one fixed array per device,
// resident until the process ends.  Host code must not pass `scratch` itself
// to a kernel (in host code the name is a stand-in, not a device address);
// noalloc_scratch looks up each device's address once and keeps it.
constexpr long NOALLOC_PARTS = LGF_NOALLOC_MAX_SITES / SITE_BLOCK;
static __device__ __align__(256) double scratch[2 * NOALLOC_PARTS];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The current device's address of `scratch` (looked up with that device
// current on the first call on it).
int noalloc_scratch(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, LGF_ERR_DEVICE, "no HIP device");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(nullptr, LGF_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, LGF_ERR_DEVICE,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LGF_OK;
}

}  // namespace

namespace lgf {
bool fft_plan_fits(const fft_plan &p) {
    constexpr size_t LDS_MAX = 160 * 1024;
    auto axis_ok = [&](const axis_plan &a) {
        return a.lds <= LDS_MAX && (a.nslice + a.B - 1) / a.B <= 65535;
    };
    if (p.xy != 2 && p.lds_xy > LDS_MAX) return false;
    if (p.xy == 2 && !(axis_ok(p.x) && axis_ok(p.y))) return false;
    if (p.zt2 && p.lds_zt2 > LDS_MAX) return false;
    if (p.rc) return p.lds <= LDS_MAX;
    return axis_ok(p.z) && axis_ok(p.t);
}
}  // namespace lgf

// =================================================================== C ABI

extern "C" {

int lgf_create(lgf_ctx **out, const int L[4], int precision, void *stream) {
    return lgf_create_group(out, L, 3, precision, stream);
}

int lgf_create_group(lgf_ctx **out, const int L[4], int nc, int precision, void *stream) {
    if (!out || !L) return fail(nullptr, LGF_ERR_ARG, "null argument");
    *out = nullptr;
    if (nc != 2 && nc != 3) return fail(nullptr, LGF_ERR_ARG, "gauge group must be SU(2) or SU(3)");
    if (!shape_ok(L))
        return fail(nullptr, LGF_ERR_ARG,
                    "unsupported lattice extent (allowed: 2^a 3^b from 2 to 256, fewer than "
                    "2^31 sites)");
    {
        const geom g0 = make_geom(L, nc);
        if (!fft_plan_fits(plan_fft<double>(g0, ZT_LDS_BUDGET, 0)) ||
            !fft_plan_fits(plan_fft<float>(g0, ZT_LDS_BUDGET, 0)))
            return fail(nullptr, LGF_ERR_ARG, "lattice extent: transform passes exceed the "
                                              "LDS or grid limits");
    }
    if (precision != LGF_FP64 && precision != LGF_MIXED)
        return fail(nullptr, LGF_ERR_ARG, "precision must be LGF_FP64 or LGF_MIXED");
    lgf_ctx *c = new (std::nothrow) lgf_ctx();
    if (!c) return fail(nullptr, LGF_ERR_OOM, "host allocation failed");
    c->g = make_geom(L, nc);
    c->precision = precision;
    c->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, LGF_ERR_DEVICE, "no HIP device");
    }
    const long V = c->g.V;
    c->nparts = site_blocks(V);
    auto alloc = [&](void **p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
    bool ok = true;
    const long S = c->g.S;
    ok = ok && alloc_links(c);
    ok = ok && alloc((void **)&c->D64[0], (size_t)c->g.nf * S * sizeof(double2));
    ok = ok && alloc((void **)&c->D64[1], (size_t)c->g.nf * S * sizeof(double2));
    // accumulated transformation (mixed): row 0 and 1 (SU(3)) or row 0 (SU(2))
    if (precision == LGF_MIXED)
        ok = ok && alloc((void **)&c->G32, (size_t)(nc == 3 ? 6 : 2) * S * sizeof(float2));
    const int nt = L[0] + L[1] + L[2] + L[3];
    ok = ok && alloc((void **)&c->tw64, nt * sizeof(double2));
    ok = ok && alloc((void **)&c->tw32, nt * sizeof(float2));
    ok = ok && alloc((void **)&c->pt64, nt * sizeof(double));
    ok = ok && alloc((void **)&c->pt32, nt * sizeof(float));
    ok = ok && alloc((void **)&c->partials, (size_t)2 * c->nparts * sizeof(double));
    ok = ok && alloc((void **)&c->status, sizeof(dev_status));
    ok = ok && alloc((void **)&c->reduce_out, 2 * sizeof(double));
    ok = ok && alloc((void **)&c->histF, HIST_CAP * sizeof(double));
    ok = ok && alloc((void **)&c->histT, HIST_CAP * sizeof(double));
    ok = ok && hipHostMalloc((void **)&c->status_host, 3 * sizeof(dev_status), 0) == hipSuccess;
    for (auto &ev : c->batch_ev)
        ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&c->reduce_host, 2 * sizeof(double), 0) == hipSuccess;
    if (!ok) {
        lgf_destroy(c);
        return fail(nullptr, LGF_ERR_OOM, "out of device memory");
    }

    auto tw64 = make_twiddles<double2>(c->g);
    auto tw32 = make_twiddles<float2>(c->g);
    long double p2max = 0;
    auto pt = make_p2_tables(c->g, p2max);
    c->p2max = (double)p2max;
    std::vector<double> pt64(pt.begin(), pt.end());
    std::vector<float> pt32(pt.begin(), pt.end());
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(c->tw64, tw64.data(), nt * sizeof(double2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->tw32, tw32.data(), nt * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->pt64, pt64.data(), nt * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->pt32, pt32.data(), nt * sizeof(float), hipMemcpyHostToDevice);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
        ncu = 0;  // no two-tile passes
    c->plan64 = plan_fft<double>(c->g, ZT_LDS_BUDGET, ncu);
    c->plan32 = plan_fft<float>(c->g, ZT_LDS_BUDGET, ncu);
    // best effort: a launch that still exceeds the limit reports its own error
    fft_set_max_lds<double>(c->g, c->plan64);
    fft_set_max_lds<float>(c->g, c->plan32);
    update_set_max_lds();
    if (e != hipSuccess) {
        std::string m = std::string("initialisation failed: ") + hipGetErrorString(e);
        lgf_destroy(c);
        return fail(nullptr, LGF_ERR_DEVICE, m);
    }
    *out = c;
    return LGF_OK;
}

void lgf_destroy(lgf_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    void *dev[] = {c->L64[0], c->L64[1], c->D64[0], c->D64[1], c->G32, c->tw64, c->tw32,
                   c->pt64, c->pt32, c->partials, c->status, c->reduce_out, c->histF, c->histT,
                   c->gaos, c->Lrot, c->Gex};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (c->status_host) (void)hipHostFree(c->status_host);
    for (auto ev : c->batch_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->reduce_host) (void)hipHostFree(c->reduce_host);
    delete c;
}

int lgf_set_acceleration(lgf_ctx *c, int on) {
    if (!c) return LGF_ERR_ARG;
    c->accelerate = on != 0;
    return LGF_OK;
}

int lgf_set_link_format(lgf_ctx *c, int nreal) {
    if (!c) return LGF_ERR_ARG;
    if (nreal != 12 && nreal != 18 && nreal != 8)
        return fail(c, LGF_ERR_ARG, "link format must be 8, 12 or 18");
    if (c->g.nc != 3) return fail(c, LGF_ERR_ARG, "link formats apply to SU(3) contexts");
    if (nreal == c->g.lf) return LGF_OK;
    if (hipSetDevice(c->device) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(c, LGF_ERR_DEVICE, "device unavailable");
    c->g.lf = nreal;
    if (!alloc_links(c)) {
        c->g.lf = 12;
        (void)alloc_links(c);  // on failure the buffers stay null; check_ctx reports it
        return fail(c, LGF_ERR_OOM, "out of device memory (links)");
    }
    return LGF_OK;
}

int lgf_set_field_precision(lgf_ctx *c, int bits) {
    if (!c) return LGF_ERR_ARG;
    if (bits != 32 && bits != 64) return fail(c, LGF_ERR_ARG, "field precision must be 32 or 64");
    c->g.ff32 = bits == 32 ? 1 : 0;
    return LGF_OK;
}

int lgf_set_exponential(lgf_ctx *c, int exact) {
    if (!c) return LGF_ERR_ARG;
    if (exact && c->g.nc == 3 && !c->Gex) {
        if (hipSetDevice(c->device) != hipSuccess ||
            hipMalloc((void **)&c->Gex, (size_t)6 * c->g.S * sizeof(double2)) != hipSuccess) {
            c->Gex = nullptr;
            return fail(c, LGF_ERR_OOM, "out of device memory (exact exponential)");
        }
    }
    c->exact_exp = exact != 0;
    return LGF_OK;
}

int lgf_set_theta_switch(lgf_ctx *c, double theta_switch) {
    if (!c || !(theta_switch > 0)) return fail(c, LGF_ERR_ARG, "theta_switch must be > 0");
    c->theta_switch = theta_switch;
    return LGF_OK;
}

static int solve(lgf_ctx *c, double *U, double alpha, double tol, int max_iter, lgf_result *res) {
    Timer tm;
    int rc = check_ctx(c);
    if (rc) return rc;
    dev_status st{};
    int n32 = 0, n64 = 0, code = ST_CONVERGED;
    int cur64 = 0;
    if (c->precision == LGF_MIXED) {
        // FP32 phase on a downcast copy; G accumulates the applied transformation
        HIPCHK(c, launch_pack_links<float>(U, c->L32[0], c->g, c->stream));
        HIPCHK(c, launch_g_identity(c->G32, c->g, c->stream));
        const double tol32 = std::max(tol, c->theta_switch);
        // the FP32 phase also ends when theta stops reaching new minima (its
        // rounding floor lies above the hand-over threshold)
        rc = run_phase<float>(c, alpha, tol32, max_iter, 0, st, FP32_STALL_SWEEPS);
        if (rc) return rc;
        n32 = st.n;
        code = st.code;
        // hand-over: U = G U0 G^dagger in FP64 (G reunitarised in FP64); for
        // SU(3) fused with the FP64 phase's first divergence
        const bool refine = code == ST_CONVERGED || code == ST_MAXITER || code == ST_STALLED;
        const bool fused = refine && c->g.nc == 3;
        if (fused) {
            HIPCHK(c, launch_status_reset(c->status, n32, c->stream));
            HIPCHK(c, launch_switch_div(c->g, acc_G(c, n32), U, c->L64[0], c->D64[0], c->partials,
                                        c->status, finp(c, true, tol, max_iter - n32, 0, 0),
                                        c->stream));
        } else {
            HIPCHK(c, launch_switch(c->g, acc_G(c, n32), U, c->L64[0], c->stream));
        }
        if (refine) {
            rc = run_phase<double>(c, alpha, tol, max_iter - n32, n32, st, 0, fused);
            if (rc) return rc;
            n64 = st.n;
            code = st.code;
            cur64 = n64 & 1;
        }
    } else {
        HIPCHK(c, launch_pack_links<double>(U, c->L64[0], c->g, c->stream));
        rc = run_phase<double>(c, alpha, tol, max_iter, 0, st);
        if (rc) return rc;
        n64 = st.n;
        code = st.code;
        cur64 = n64 & 1;
    }
    HIPCHK(c, launch_unpack_links(c->L64[cur64], U, c->g, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->hist_len = n32 + n64 + 1;
    const int out = status_to_code(code);
    if (res) {
        res->iterations = n32 + n64;
        res->fp32_iterations = n32;
        res->status = out;
        res->F = st.F;
        res->theta = st.theta;
        res->seconds = tm.seconds();
    }
    if (out != LGF_OK) {
        const char *m = out == LGF_NOT_CONVERGED ? "max_iter reached before theta < tol"
                        : out == LGF_ERR_NONFINITE ? "theta became non-finite"
                                                   : "theta rising: the iteration diverges";
        c->err = m;
    }
    return out;
}

int lgf_fix(lgf_ctx *c, double *U, double alpha, double theta_tol, int max_iter, lgf_result *res) {
    if (!c) return LGF_ERR_ARG;
    if (!U) return fail(c, LGF_ERR_ARG, "U is NULL");
    if (!(alpha > 0) || !(theta_tol > 0) || max_iter < 0)
        return fail(c, LGF_ERR_ARG, "need alpha > 0, theta_tol > 0, max_iter >= 0");
    return solve(c, U, alpha, theta_tol, max_iter, res);
}

int lgf_iterate(lgf_ctx *c, double *U, double alpha, int n_iter, lgf_result *res) {
    if (!c) return LGF_ERR_ARG;
    if (!U) return fail(c, LGF_ERR_ARG, "U is NULL");
    if (!(alpha > 0) || n_iter < 0) return fail(c, LGF_ERR_ARG, "need alpha > 0, n_iter >= 0");
    Timer tm;
    int rc = check_ctx(c);
    if (rc) return rc;
    dev_status st{};
    int n32 = 0, n64 = 0, cur64 = 0;
    if (c->precision == LGF_MIXED) {
        HIPCHK(c, launch_pack_links<float>(U, c->L32[0], c->g, c->stream));
        HIPCHK(c, launch_g_identity(c->G32, c->g, c->stream));
        rc = run_phase<float>(c, alpha, 0.0, n_iter, 0, st);
        if (rc) return rc;
        n32 = st.n;
        HIPCHK(c, launch_switch(c->g, acc_G(c, n32), U, c->L64[0], c->stream));
    } else {
        HIPCHK(c, launch_pack_links<double>(U, c->L64[0], c->g, c->stream));
        rc = run_phase<double>(c, alpha, 0.0, n_iter, 0, st);
        if (rc) return rc;
        n64 = st.n;
        cur64 = n64 & 1;
    }
    HIPCHK(c, launch_unpack_links(c->L64[cur64], U, c->g, c->stream));
    double F = st.F, th = st.theta;
    if (c->precision == LGF_MIXED) {
        rc = eval_links64(c, U, F, th);
        if (rc) return rc;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->hist_len = n32 + n64 + 1;
    int out = (st.code == ST_NONFINITE) ? LGF_ERR_NONFINITE : LGF_OK;
    if (res) {
        res->iterations = n32 + n64;
        res->fp32_iterations = n32;
        res->status = out;
        res->F = F;
        res->theta = th;
        res->seconds = tm.seconds();
    }
    return out;
}

int lgf_functional(lgf_ctx *c, const double *U, const double *g, double *F) {
    if (!c) return LGF_ERR_ARG;
    if (g && c->g.nc != 3) return fail(c, LGF_ERR_ARG, "F_U[g] with g is available for SU(3) only");
    if (!U || !F) return fail(c, LGF_ERR_ARG, "null argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!g) {
        double th;
        return eval_links64(c, U, *F, th);
    }
    HIPCHK(c, launch_pack_links<double>(U, c->L64[0], g12(c), c->stream));
    HIPCHK(c, launch_functional_g(c->g, c->L64[0], g, c->partials, c->stream));
    double A, B;
    rc = sum_partials(c, A, B);
    if (rc) return rc;
    *F = A * normF(c);
    return LGF_OK;
}

int lgf_theta(lgf_ctx *c, const double *U, double *theta) {
    if (!c) return LGF_ERR_ARG;
    if (!U || !theta) return fail(c, LGF_ERR_ARG, "null argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    double F;
    return eval_links64(c, U, F, *theta);
}

int lgf_plaquette(lgf_ctx *c, const double *U, double *P) {
    if (!c) return LGF_ERR_ARG;
    if (c->g.nc != 3) return fail(c, LGF_ERR_ARG, "the plaquette is available for SU(3) only");
    if (!U || !P) return fail(c, LGF_ERR_ARG, "null argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    HIPCHK(c, launch_pack_links<double>(U, c->L64[0], g12(c), c->stream));
    HIPCHK(c, launch_plaquette(c->g, c->L64[0], c->partials, c->stream));
    double A, B;
    rc = sum_partials(c, A, B);
    if (rc) return rc;
    *P = A / (6.0 * 3.0 * (double)c->g.V);
    return LGF_OK;
}

int lgf_divergence(lgf_ctx *c, const double *U, double *Delta) {
    if (!c) return LGF_ERR_ARG;
    if (c->g.nc != 3) return fail(c, LGF_ERR_ARG, "lgf_divergence is available for SU(3) only");
    if (!U || !Delta) return fail(c, LGF_ERR_ARG, "null argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    HIPCHK(c, launch_pack_links<double>(U, c->L64[0], g12(c), c->stream));
    HIPCHK(c, launch_status_reset(c->status, 0, c->stream));
    HIPCHK(c, launch_div_reduce<double>(g12(c), c->L64[0], c->D64[0], c->partials, c->status,
                                        finp(c, false), c->stream));
    HIPCHK(c, launch_matrix_from_field(c->D64[0], Delta, c->g.V, c->g.S, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGF_OK;
}

int lgf_fourier_accelerate(lgf_ctx *c, const double *D, double *LD) {
    if (!c) return LGF_ERR_ARG;
    if (c->g.nc != 3) return fail(c, LGF_ERR_ARG, "lgf_fourier_accelerate is available for SU(3) only");
    if (!D || !LD) return fail(c, LGF_ERR_ARG, "null argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    HIPCHK(c, launch_status_reset(c->status, 0, c->stream));
    HIPCHK(c, launch_field_from_matrix(D, c->D64[0], c->g.V, c->g.S, c->stream));
    HIPCHK(c, launch_fft_xy<double>(c->g, c->D64[0], -1, c->tw64, c->plan64, c->status,
                                    c->stream));
    HIPCHK(c, launch_fft_zt<double>(c->g, c->D64[0], 0, c->tw64, c->pt64,
                                    c->p2max / (double)c->g.V, c->plan64, c->status, c->stream));
    HIPCHK(c, launch_fft_xy<double>(c->g, c->D64[0], +1, c->tw64, c->plan64, c->status,
                                    c->stream));
    HIPCHK(c, launch_matrix_from_field(c->D64[0], LD, c->g.V, c->g.S, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGF_OK;
}

int lgf_fft4d(lgf_ctx *c, double *fields, int sign) {
    if (!c) return LGF_ERR_ARG;
    if (c->g.nc != 3) return fail(c, LGF_ERR_ARG, "lgf_fft4d is available for SU(3) only");
    if (!fields || (sign != 1 && sign != -1)) return fail(c, LGF_ERR_ARG, "bad argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    double2 *F = reinterpret_cast<double2 *>(fields);
    const long V = c->g.V, S = c->g.S;
    double2 *W = c->D64[0];
    const size_t row = (size_t)V * sizeof(double2);
    HIPCHK(c, launch_status_reset(c->status, 0, c->stream));
    if (sign < 0) {
        // caller layout (stride V) -> work buffer (stride S), transform, natural order back
        HIPCHK(c, hipMemcpy2DAsync(W, S * sizeof(double2), F, row, row, 4,
                                   hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, launch_fft_xy<double>(c->g, W, -1, c->tw64, c->plan64, c->status, c->stream));
        HIPCHK(c, launch_fft_zt<double>(c->g, W, -1, c->tw64, c->pt64, 0.0, c->plan64, c->status,
                                        c->stream));
        HIPCHK(c, launch_reorder_fields(c->g, W, S, F, V, 1, c->stream));
    } else {
        HIPCHK(c, launch_reorder_fields(c->g, F, V, W, S, 0, c->stream));
        HIPCHK(c, launch_fft_zt<double>(c->g, W, +1, c->tw64, c->pt64, 0.0, c->plan64, c->status,
                                        c->stream));
        HIPCHK(c, launch_fft_xy<double>(c->g, W, +1, c->tw64, c->plan64, c->status, c->stream));
        HIPCHK(c, hipMemcpy2DAsync(F, row, W, S * sizeof(double2), row, 4,
                                   hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGF_OK;
}

int lgf_functional_omega(lgf_ctx *c, const double *U, const double *omega, double *F) {
    if (!c) return LGF_ERR_ARG;
    if (c->g.nc != 3) return fail(c, LGF_ERR_ARG, "the omega parametrisation is available for SU(3) only");
    if (!U || !omega || !F) return fail(c, LGF_ERR_ARG, "null argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = ensure_diff_scratch(c))) return rc;
    HIPCHK(c, launch_expm_sites(omega, c->gaos, c->g.V, c->stream));
    return lgf_functional(c, U, c->gaos, F);
}

int lgf_functional_omega_grad(lgf_ctx *c, const double *U, const double *omega, double *F,
                              double *dF) {
    if (!c) return LGF_ERR_ARG;
    if (c->g.nc != 3) return fail(c, LGF_ERR_ARG, "the omega parametrisation is available for SU(3) only");
    if (!U || !omega || !F || !dF) return fail(c, LGF_ERR_ARG, "null argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = ensure_diff_scratch(c))) return rc;
    HIPCHK(c, launch_expm_sites(omega, c->gaos, c->g.V, c->stream));
    HIPCHK(c, launch_pack_links<double>(U, c->L64[0], g12(c), c->stream));
    HIPCHK(c, launch_rotate_links(c->g, c->L64[0], c->gaos, c->Lrot, c->stream));
    HIPCHK(c, launch_status_reset(c->status, 0, c->stream));
    HIPCHK(c, launch_div_reduce<double>(g12(c), c->Lrot, c->D64[0], c->partials, c->status,
                                        finp(c, false), c->stream));
    double A, B;
    rc = sum_partials(c, A, B);
    if (rc) return rc;
    *F = A * normF(c);
    HIPCHK(c, launch_omega_grad(c->g, c->D64[0], omega, dF, normF(c), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGF_OK;
}

int lgf_theta_grad(lgf_ctx *c, const double *U, const double *eps, double *theta, double *dtheta) {
    if (!c) return LGF_ERR_ARG;
    if (c->g.nc != 3) return fail(c, LGF_ERR_ARG, "the theta gradient is available for SU(3) only");
    if (!U || !theta) return fail(c, LGF_ERR_ARG, "null argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    if ((rc = ensure_diff_scratch(c))) return rc;
    HIPCHK(c, launch_pack_links<double>(U, c->L64[0], g12(c), c->stream));
    const void *Lw = c->L64[0];
    if (eps) {
        HIPCHK(c, launch_expm_sites(eps, c->gaos, 4 * c->g.V, c->stream));
        HIPCHK(c, launch_left_multiply_links(c->L64[0], c->gaos, c->Lrot, c->g.V, c->g.S, c->stream));
        Lw = c->Lrot;
    }
    HIPCHK(c, launch_status_reset(c->status, 0, c->stream));
    HIPCHK(c, launch_div_reduce<double>(g12(c), Lw, c->D64[0], c->partials, c->status,
                                        finp(c, false), c->stream));
    double A, B;
    rc = sum_partials(c, A, B);
    if (rc) return rc;
    *theta = B * normT(c);
    if (dtheta) {
        HIPCHK(c, launch_theta_grad(c->g, Lw, c->D64[0], eps, dtheta, normT(c), c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return LGF_OK;
}

int lgf_profile(lgf_ctx *c, const double *U, double alpha, int n_iter, double *kernel_ms) {
    if (!c) return LGF_ERR_ARG;
    if (!U || !kernel_ms || n_iter < 1 || !(alpha > 0))
        return fail(c, LGF_ERR_ARG, "need U, kernel_ms, n_iter >= 1, alpha > 0");
    int rc = check_ctx(c);
    if (rc) return rc;
    return c->precision == LGF_MIXED ? profile_impl<float>(c, U, alpha, n_iter, kernel_ms)
                                     : profile_impl<double>(c, U, alpha, n_iter, kernel_ms);
}

int lgf_history(lgf_ctx *c, double *F, double *theta, int cap, int *count) {
    if (!c || !count || cap < 0) return fail(c, LGF_ERR_ARG, "bad argument");
    int rc = check_ctx(c);
    if (rc) return rc;
    const int n = std::min(std::min(cap, c->hist_len), HIST_CAP);
    if (n > 0 && F)
        HIPCHK(c, hipMemcpy(F, c->histF, n * sizeof(double), hipMemcpyDeviceToHost));
    if (n > 0 && theta)
        HIPCHK(c, hipMemcpy(theta, c->histT, n * sizeof(double), hipMemcpyDeviceToHost));
    *count = n;
    return LGF_OK;
}

int lgf_measure_noalloc(const int L[4], const double *U, double *out, void *stream) {
    if (!L || !U || !out) return fail(nullptr, LGF_ERR_ARG, "null argument");
    if (!shape_ok(L))
        return fail(nullptr, LGF_ERR_ARG, "unsupported lattice extent");
    const geom g = make_geom(L, 3);
    if (g.V > LGF_NOALLOC_MAX_SITES)
        return fail(nullptr, LGF_ERR_ARG,
                    "lattice of " + std::to_string(g.V) + " sites exceeds the " +
                        std::to_string((long)LGF_NOALLOC_MAX_SITES) +
                        " sites of the fixed scratch array");
    double *partials = nullptr;
    const int rc = noalloc_scratch(&partials);
    if (rc) return rc;
    const hipError_t e =
        launch_measure_aos(g, U, partials, out, 1.0 / (4.0 * 3.0 * (double)g.V),
                           1.0 / (3.0 * (double)g.V), static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(nullptr, LGF_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return LGF_OK;
}

const char *lgf_last_error(const lgf_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
