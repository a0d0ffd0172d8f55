// HIP kernels of the Fourier-accelerated Landau gauge-fixing sweep (gfx950).
//
// One sweep (one gauge update) is four launches plus a one-block finalize:
//   fft_xy(-1)  2D transform over the contiguous (x, y) planes, in place
//   fft_zt(0)   2D transform over (z, t), scaling by p2max/(V p2), inverse
//               (z, t) transform, in place: tiles of W consecutive xy-sites
//   fft_xy(+1)  inverse (x, y) transform -> L Delta
//   update      g = reunit(1 + alpha/2 L Delta) at x and its 8 neighbours,
//               U'_mu(x) = g(x) U_mu(x) g(x+mu)^dagger (written), and the next
//               Delta(x) from U'_mu(x) and the recomputed U'_mu(x-mu), with
//               block partial sums of F and theta
//   finalize    fixed-order sum of the partials, stopping test
// Links are double-buffered (the update reads U_mu(x-mu) of other threads),
// as are the Fourier fields.  The FP32 sweeps of an SU(3) mixed solve store
// no links: their inverse (x, y) pass (or k_gauge_acc after it) turns L Delta
// into G <- g G, double-buffered, and the update forms G U0 G^dagger from the
// constant input copy U0.
#include <type_traits>

#include "common.hpp"

namespace lgf {

// ---------------------------------------------------------------------------
// layout conversion
// ---------------------------------------------------------------------------

// A caller link (complex128 AoS, rows 0,1; all three rows for the 18-real
// format) as an SU(3) matrix of type T.
template <class T, int LF> __device__ __forceinline__ mat3<T> aos_link(const double2 *__restrict__ u) {
    constexpr int NIN = LF == 18 ? 9 : 6;
    mat3<T> m;
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
        const double2 v = u[k];
        m.e[k / 3][k % 3] = mk<T>((T)v.x, (T)v.y);
    }
    if constexpr (LF != 18) rebuild_row2(m);
    return m;
}

// complex128 [4][V][3][3] -> SoA of type T in link format LF
template <class T, int LF>
__global__ void __launch_bounds__(256) k_pack_links(const double2 *__restrict__ U,
                                                    vec2_t<T> *__restrict__ L, long V, long S) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = (int)(i / V);
    const long s = i - (long)mu * V;
    cpx<T> sl[LF / 2];
    link_to_slots<T, LF>(aos_link<T, LF>(U + i * 9), sl);
#pragma unroll
    for (int k = 0; k < LF / 2; ++k) st<T>(L + ((long)mu * (LF / 2) + k) * S + s, sl[k]);
}

template <int LF>
__global__ void __launch_bounds__(256) k_unpack_links(const double2 *__restrict__ L,
                                                      double2 *__restrict__ U, long V, long S) {
    // The block's 256 links are assembled in LDS and written out as one
    // contiguous run (consecutive lanes on consecutive 16-byte entries), not
    // as 144-byte strided pieces per lane.
    __shared__ double2 buf[256 * 9];
    const long i0 = (long)blockIdx.x * 256, i = i0 + threadIdx.x;
    const long n = min(4 * V - i0, 256L);
    if (i < 4 * V) {
        const int mu = (int)(i / V);
        const long s = i - (long)mu * V;
        const mat3<double> m = load_link<double, LF>(L, S, mu, s);
#pragma unroll
        for (int k = 0; k < 9; ++k)
            buf[threadIdx.x * 9 + k] = make_double2(m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im);
    }
    __syncthreads();
    double2 *u = U + i0 * 9;
    for (int e = threadIdx.x; e < n * 9; e += 256) u[e] = buf[e];
}

// anti-hermitian traceless matrix field (AoS 3x3 complex128) <-> 4 Fourier fields
__global__ void k_field_from_matrix(const double2 *__restrict__ M, double2 *__restrict__ D, long V,
                                    long S) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const double2 *m = M + s * 9;
    D[s] = m[1];
    D[S + s] = m[2];
    D[2 * S + s] = m[5];
    D[3 * S + s] = make_double2(m[0].y, m[4].y);
}

__global__ void k_matrix_from_field(const double2 *__restrict__ D, double2 *__restrict__ M, long V,
                                    long S) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    const double2 f0 = D[s], f1 = D[S + s], f2 = D[2 * S + s], f3 = D[3 * S + s];
    double2 *m = M + s * 9;
    m[0] = make_double2(0.0, f3.x);
    m[1] = f0;
    m[2] = f1;
    m[3] = make_double2(-f0.x, f0.y);
    m[4] = make_double2(0.0, f3.y);
    m[5] = f2;
    m[6] = make_double2(-f1.x, f1.y);
    m[7] = make_double2(-f2.x, f2.y);
    m[8] = make_double2(0.0, -(f3.x + f3.y));
}

// ---------------------------------------------------------------------------
// finalize: fixed-order sum of block partials and the stopping test
// ---------------------------------------------------------------------------

constexpr int FIN_BLOCK = 1024;

template <int NT>
__device__ __forceinline__ void fixed_order_sum(const double *__restrict__ partials, int nparts,
                                                double &A, double &B) {
    // thread t adds pairs t, t + NT, t + 2 NT, ... in that order; four 16-byte
    // loads are in flight per step
    const double2 *p2 = reinterpret_cast<const double2 *>(partials);
    double a = 0, b = 0;
    int i = threadIdx.x;
    for (; i + 3 * NT < nparts; i += 4 * NT) {
        const double2 v0 = p2[i], v1 = p2[i + NT], v2 = p2[i + 2 * NT], v3 = p2[i + 3 * NT];
        a += v0.x;
        b += v0.y;
        a += v1.x;
        b += v1.y;
        a += v2.x;
        b += v2.y;
        a += v3.x;
        b += v3.y;
    }
    for (; i < nparts; i += NT) {
        const double2 v = p2[i];
        a += v.x;
        b += v.y;
    }
    __shared__ double sa[NT], sb[NT];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sa[threadIdx.x] += sa[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    A = sa[0];
    B = sb[0];
}

// F = A normF, theta = B normT; history, stopping test (one thread)
__device__ __forceinline__ void finalize_state(double A, double B, dev_status *status,
                                               const fin_params &fp) {
    const double F = A * fp.normF, th = B * fp.normT;
    dev_status st = *status;
    if (fp.increment) st.n += 1;
    const int h = st.hist_base + st.n;
    if (h < fp.hist_cap) {
        fp.histF[h] = F;
        fp.histT[h] = th;
    }
    st.F = F;
    st.theta = th;
    if (!isfinite(th) || !isfinite(F)) {
        st.done = 1;
        st.code = ST_NONFINITE;
    } else if (th < fp.tol) {
        st.done = 1;
        st.code = ST_CONVERGED;
    } else if (st.n >= fp.max_iter) {
        st.done = 1;
        st.code = ST_MAXITER;
    } else if (fp.tol > 0) {
        // a solve (tol > 0) also stops when theta diverges or stalls; a fixed
        // count of sweeps (tol == 0) runs them all
        st.rises = (st.n > 0 && th > st.theta_prev) ? st.rises + 1 : 0;
        st.since_min = (st.n == 0 || th < st.theta_min) ? 0 : st.since_min + 1;
        if (st.rises >= DIVERGE_RISES && th > DIVERGE_GROWTH * st.theta_min) {
            st.done = 1;
            st.code = ST_DIVERGING;
        } else if (fp.stall > 0 && st.since_min >= fp.stall) {
            st.done = 1;
            st.code = ST_STALLED;
        }
    }
    st.theta_prev = th;
    st.theta_min = (st.n == 0 || th < st.theta_min) ? th : st.theta_min;
    *status = st;
}

// ---------------------------------------------------------------------------
// divergence and reductions of given links (first sweep of a solve)
// ---------------------------------------------------------------------------

// TF: real type of the Fourier field (T, or float for FP64 sweeps whose field
// is held in FP32)
// Delta(x) of the links link(mu, site), packed into the 4 field entries f;
// tr = sum_mu Re Tr U_mu(x); returns Tr[Delta Delta^dagger].
template <class T, class LinkFn>
__device__ __forceinline__ T divergence_at(const geom &g, long s, LinkFn link, cpx<T> (&f)[4],
                                           T &tr) {
    const nbr n = neighbours(g, s);
    xacc<T> X;
    xacc_zero(X);
    tr = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        mat3<T> u = link(mu, s);
        tr += retrace(u);
        xacc_add(X, u, T(-1));
        mat3<T> um = link(mu, n.m[mu]);
        xacc_add(X, um, T(1));
    }
    return delta_pack(X, f[0], f[1], f[2], f[3]);
}

template <class T, class TF, int LF>
__global__ void __launch_bounds__(SITE_BLOCK)
    k_div_reduce(geom g, const vec2_t<T> *__restrict__ L, vec2_t<TF> *__restrict__ D,
                 double *__restrict__ partials, const dev_status *__restrict__ status) {
    if (status->done) return;
    const long s = block_site(g, blockIdx.x, gridDim.x, threadIdx.x);
    double fs = 0, ts = 0;
    if (s < g.V) {
        cpx<T> f[4];
        T tr;
        ts = (double)divergence_at<T>(
            g, s, [&](int mu, long x) { return load_link<T, LF>(L, g.S, mu, x); }, f, tr);
        fs = (double)tr;
#pragma unroll
        for (int k = 0; k < 4; ++k) st<TF>(D + k * g.S + s, cvt<TF>(f[k]));
    }
    block_sum2<SITE_BLOCK>(fs, ts, partials, blockIdx.x);
}

// k_div_reduce<double, double, 2> reading the caller's AoS links directly
// (rows 0,1; row 2 rebuilt as a 12-real load does) and storing no field.
__global__ void __launch_bounds__(SITE_BLOCK)
    k_measure_aos(geom g, const double2 *__restrict__ U, double *__restrict__ partials) {
    const long s = block_site(g, blockIdx.x, gridDim.x, threadIdx.x);
    double fs = 0, ts = 0;
    if (s < g.V) {
        auto link = [&](int mu, long x) {
            mat3<double> m;
            const double2 *u = U + ((long)mu * g.V + x) * 9;
#pragma unroll
            for (int k = 0; k < 6; ++k) m.e[k / 3][k % 3] = mk<double>(u[k].x, u[k].y);
            rebuild_row2(m);
            return m;
        };
        cpx<double> f[4];
        double tr;
        ts = divergence_at<double>(g, s, link, f, tr);
        fs = tr;
    }
    block_sum2<SITE_BLOCK>(fs, ts, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// fused update + next divergence
// ---------------------------------------------------------------------------

// GPRE: each site's transformation was computed beforehand and is read as
// rows 0,1 from GX (6 entries per site) instead of being formed from L Delta:
// g = exp((alpha/2) L Delta) of the exact step (k_gauge_exp), or the
// accumulated G of the FP32 sweeps (k_gauge_acc), whose links G U0 G^dagger
// come from the constant input copy U0 in Lin.  STORE: write the new links to
// Lout (the FP32 sweeps keep U0 and G instead).
template <class T, class TF, bool GPRE, int LF, bool STORE>
__global__ void __launch_bounds__(SITE_BLOCK)
    k_update(geom g, const vec2_t<T> *__restrict__ Lin, vec2_t<T> *__restrict__ Lout,
             const vec2_t<TF> *__restrict__ LD, const vec2_t<T> *__restrict__ GX,
             vec2_t<TF> *__restrict__ Dout, T c, double *__restrict__ partials,
             const dev_status *__restrict__ status) {
    if (status->done) return;
    const long s = block_site(g, blockIdx.x, gridDim.x, threadIdx.x);
    double fs = 0, ts = 0;
    if (s < g.V) {
        const nbr n = neighbours(g, s);
        // Eight half-steps h = 2 mu + b: b = 0 transforms the link U_mu(x)
        // with g(x+mu), b = 1 the link U_mu(x-mu) with g(x-mu).  Each needs
        // the 4 field entries of g's site (6 entries of g itself when GPRE)
        // and the LF/2 stored slots of the link; the loads of half-step h+1 are issued before
        // half-step h is computed (software pipelining), so every wave keeps
        // the next memory round trip in flight.
        constexpr int NG = GPRE ? 6 : 4;
        struct half {
            cpx<T> f[NG], u[LF / 2];
        };
        auto load_g = [&](long x, cpx<T> (&f)[NG]) {
#pragma unroll
            for (int k = 0; k < NG; ++k) {
                if constexpr (GPRE) f[k] = ld<T>(GX + (long)k * g.S + x);
                else f[k] = cvt<T>(ld<TF>(LD + (long)k * g.S + x));
            }
        };
        auto make_g = [&](const cpx<T> (&f)[NG]) {
            mat3<T> m;
            if constexpr (GPRE) {
#pragma unroll
                for (int k = 0; k < 6; ++k) m.e[k / 3][k % 3] = f[k];
                rebuild_row2(m);
            } else {
                m = gauge_from_entries<T>(f[0], f[1], f[2], f[3], c);
            }
            return m;
        };
        auto fetch = [&](int h, half &d) {
            const int mu = h >> 1;
            const long sf = (h & 1) ? n.m[mu] : n.p[mu];
            const long sl = (h & 1) ? n.m[mu] : s;
            load_g(sf, d.f);
            const vec2_t<T> *lp = Lin + (long)mu * (LF / 2) * g.S + sl;
#pragma unroll
            for (int k = 0; k < LF / 2; ++k) d.u[k] = ld<T>(lp + (long)k * g.S);
        };
        half d[2];
        cpx<T> own[NG];
        load_g(s, own);
        fetch(0, d[0]);
        const mat3<T> g0 = make_g(own);
        xacc<T> X;
        xacc_zero(X);
        T tr = 0;
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            if (h < 7) fetch(h + 1, d[(h + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            const half &cur = d[h & 1];
            const mat3<T> gn = make_g(cur.f);
            const mat3<T> u = link_from_slots<T, LF>(cur.u);
            constexpr int PR = product_rows<LF>();
            if ((h & 1) == 0) {
                const mat3<T> un = mul_abcd<PR>(g0, u, gn);  // g(x) U_mu(x) g(x+mu)^+
                if constexpr (STORE) store_link<T, LF>(Lout, g.S, h >> 1, s, un);
                tr += retrace(un);
                xacc_add(X, un, T(-1));
            } else {
                const mat3<T> umn = mul_abcd<PR>(gn, u, g0);  // g(x-mu) U_mu(x-mu) g(x)^+
                xacc_add(X, umn, T(1));
            }
        }
        cpx<T> f0, f1, f2, f3;
        ts = (double)delta_pack(X, f0, f1, f2, f3);
        fs = (double)tr;
        st_stream<TF>(Dout + s, cvt<TF>(f0));
        st_stream<TF>(Dout + g.S + s, cvt<TF>(f1));
        st_stream<TF>(Dout + 2 * g.S + s, cvt<TF>(f2));
        st_stream<TF>(Dout + 3 * g.S + s, cvt<TF>(f3));
    }
    block_sum2<SITE_BLOCK>(fs, ts, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// FP32 sweeps of an SU(3) mixed solve with the links shared through LDS
// ---------------------------------------------------------------------------

// Every link U_mu(x) enters two divergences: with sign - at x and with sign +
// at x + mu, so k_update forms each link twice.  The divergence is linear in
// the links through P(M): the off-diagonal differences M_ij - conj(M_ji)
// (i < j) and the traceless part of 2 Im M_ii, 8 reals, in the order of the 4
// Fourier-field entries.  This kernel forms the 4 links leaving each site,
// keeps their P in LDS and takes the links arriving from x - mu from LDS when
// x - mu is in the block, forming them again otherwise.  A block holds
// UPDS_XY consecutive xy-sites at UPDS_T consecutive t and one z: the x
// neighbour is in the block whenever UPDS_XY is a multiple of Lx, the y
// neighbour except in the block's first xy-row, the t neighbour except at
// its first t, the z neighbour never.  FP32 arithmetic as in k_update; the
// per-link projections change the rounding order of the sums, not the
// quantities.  Partial sums go out per group of SITE_BLOCK threads, so the
// finalize reads the same number of partials as after k_update.
// Blocks of 128 xy-sites x 4 t (512 threads, 64 KB of LDS) let two blocks
// share a compute unit, so that one block's loads overlap the other's
// arithmetic: 73 against 82 us at 32^4 and 797 against 828 us at 48^3 x 96
// for one block of 256 x 4 (or 256 x 2: 74 / 848 us; 128 x 2: 73 / 855 us).
constexpr int UPDS_XY = 128, UPDS_T = 4, UPDS_THREADS = UPDS_XY * UPDS_T;
constexpr size_t UPDS_LDS = (size_t)8 * 4 * UPDS_THREADS * sizeof(float);

inline bool update_shared_ok(const geom &g) {
    const long Lxy = (long)g.Lx * g.Ly;
    return g.nc == 3 && g.lf == 12 && Lxy % UPDS_XY == 0 && g.Lt % UPDS_T == 0;
}

// a += sgn * P(m)
template <class T> LGF_HD void proj_add(T (&a)[8], const mat3<T> &m, T sgn) {
    a[0] += sgn * (m.e[0][1].re - m.e[1][0].re);
    a[1] += sgn * (m.e[0][1].im + m.e[1][0].im);
    a[2] += sgn * (m.e[0][2].re - m.e[2][0].re);
    a[3] += sgn * (m.e[0][2].im + m.e[2][0].im);
    a[4] += sgn * (m.e[1][2].re - m.e[2][1].re);
    a[5] += sgn * (m.e[1][2].im + m.e[2][1].im);
    const T d0 = T(2) * m.e[0][0].im, d1 = T(2) * m.e[1][1].im, d2 = T(2) * m.e[2][2].im;
    const T tr = (d0 + d1 + d2) * T(1.0 / 3.0);
    a[6] += sgn * (d0 - tr);
    a[7] += sgn * (d1 - tr);
}

// P(m) alone
template <class T> LGF_HD void proj_of(T (&a)[8], const mat3<T> &m) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = T(0);
    proj_add(a, m, T(1));
}

// block sum of two doubles per group of NG threads into partials[2 * (slot0 + group) + {0,1}]
template <int NT, int NG>
__device__ __forceinline__ void group_sum2(double a, double b, double *partials, int slot0) {
    static_assert(NT % NG == 0 && NG % 64 == 0, "wave64 groups");
    __shared__ double sa[NT / 64], sb[NT / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x % NG == 0) {
        const int w0 = threadIdx.x >> 6;
        double A = 0, B = 0;
#pragma unroll
        for (int i = 0; i < NG / 64; ++i) {
            A += sa[w0 + i];
            B += sb[w0 + i];
        }
        const int slot = slot0 + threadIdx.x / NG;
        partials[2 * slot] = A;
        partials[2 * slot + 1] = B;
    }
}

// four waves per SIMD: two blocks per compute unit (at most 128 VGPRs)
__global__ void __launch_bounds__(UPDS_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
    k_update_shared32(geom g, const float2 *__restrict__ Lin, const float2 *__restrict__ GX,
                      float2 *__restrict__ Dout, double *__restrict__ partials,
                      const dev_status *__restrict__ status) {
    using T = float;
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    T *P = reinterpret_cast<T *>(smem_raw);  // P[(k * 4 + mu) * UPDS_THREADS + i]
    // block -> (z fastest, then the xy group, then the t group); XCDs walk
    // contiguous ranges
    const int B = xcd_block(blockIdx.x, gridDim.x);
    const unsigned Lxy = (unsigned)g.Lx * (unsigned)g.Ly, ngxy = Lxy / UPDS_XY;
    const unsigned z = (unsigned)B % (unsigned)g.Lz, r = (unsigned)B / (unsigned)g.Lz;
    const unsigned xy0 = (r % ngxy) * UPDS_XY, t0 = (r / ngxy) * UPDS_T;
    const int i = threadIdx.x;  // local index: (t - t0) * UPDS_XY + (xy - xy0)
    const unsigned xy = xy0 + (unsigned)i % UPDS_XY, t = t0 + (unsigned)i / UPDS_XY;
    const unsigned s = xy + Lxy * (z + (unsigned)g.Lz * t);
    const unsigned x = xy % (unsigned)g.Lx, y = (xy / (unsigned)g.Lx) % (unsigned)g.Ly;
    const unsigned Lx = g.Lx, Ly = g.Ly, Lz = g.Lz, Lt = g.Lt, sz = Lxy, st = Lxy * Lz;
    // neighbour s + mu (fwd) or s - mu, periodic, in 32-bit arithmetic (V < 2^31)
    auto nb = [&](int mu, bool fwd) -> unsigned {
        if (mu == 0) return fwd ? (x == Lx - 1 ? s - (Lx - 1) : s + 1) : (x == 0 ? s + (Lx - 1) : s - 1);
        if (mu == 1)
            return fwd ? (y == Ly - 1 ? s - (Ly - 1) * Lx : s + Lx) : (y == 0 ? s + (Ly - 1) * Lx : s - Lx);
        if (mu == 2)
            return fwd ? (z == Lz - 1 ? s - (Lz - 1) * sz : s + sz) : (z == 0 ? s + (Lz - 1) * sz : s - sz);
        return fwd ? (t == Lt - 1 ? s - (Lt - 1) * st : s + st) : (t == 0 ? s + (Lt - 1) * st : s - st);
    };
    const long S = g.S;
    auto load_g = [&](unsigned q, cpx<T> (&f)[6]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) f[k] = ld<T>(GX + (long)k * S + q);
    };
    auto make_g = [&](const cpx<T> (&f)[6]) {
        mat3<T> m;
#pragma unroll
        for (int k = 0; k < 6; ++k) m.e[k / 3][k % 3] = f[k];
        rebuild_row2(m);
        return m;
    };
    struct half {
        cpx<T> f[6], u[6];
    };
    // h = 2 mu + b as in k_update: b = 0 the link leaving x, b = 1 the one arriving from x - mu
    auto fetch = [&](int h, half &d) {
        const int mu = h >> 1;
        const unsigned sf = nb(mu, (h & 1) == 0);
        const unsigned sl = (h & 1) ? sf : s;
        load_g(sf, d.f);
        const float2 *lp = Lin + (long)mu * 6 * S + sl;
#pragma unroll
        for (int k = 0; k < 6; ++k) d.u[k] = ld<T>(lp + (long)k * S);
    };
    cpx<T> own[6];
    load_g(s, own);
    half d[2];
    fetch(0, d[0]);
    const mat3<T> g0 = make_g(own);
    T X[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) X[k] = T(0);
    T tr = 0;
    // links leaving x: U_mu(x) = g(x) U0_mu(x) g(x+mu)^+; the z link arriving
    // from x - z (never in the block) is fetched during the last of them
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        fetch(mu < 3 ? 2 * (mu + 1) : 5, d[(mu + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        const half &cur = d[mu & 1];
        const mat3<T> un = mul_abcd<2>(g0, link_from_slots<T, 12>(cur.u), make_g(cur.f));
        tr += retrace(un);
        T pm[8];
        proj_of(pm, un);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            P[(k * 4 + mu) * UPDS_THREADS + i] = pm[k];
            X[k] -= pm[k];
        }
    }
    // the z link arriving from x - z: g(x-z) U0_z(x-z) g(x)^+
    {
        const half &cur = d[0];
        const mat3<T> umn = mul_abcd<2>(make_g(cur.f), link_from_slots<T, 12>(cur.u), g0);
        proj_add(X, umn, T(1));
    }
    __syncthreads();
    // x, y, t links arriving from x - mu: from LDS inside the block
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        if (mu == 2) continue;
        unsigned txy = xy, tt = t;
        if (mu == 0) txy = x == 0 ? xy + Lx - 1 : xy - 1;
        if (mu == 1) txy = y == 0 ? xy + (Ly - 1) * Lx : xy - Lx;
        if (mu == 3) tt = t == 0 ? Lt - 1 : t - 1;
        const unsigned lx = txy - xy0, lt = tt - t0;
        if (lx < (unsigned)UPDS_XY && lt < (unsigned)UPDS_T) {
            const int j = (int)(lt * UPDS_XY + lx);
#pragma unroll
            for (int k = 0; k < 8; ++k) X[k] += P[(k * 4 + mu) * UPDS_THREADS + j];
        } else {
            half e;
            fetch(2 * mu + 1, e);
            const mat3<T> umn = mul_abcd<2>(make_g(e.f), link_from_slots<T, 12>(e.u), g0);
            proj_add(X, umn, T(1));
        }
    }
    const cpx<T> f0 = mk<T>(X[0], X[1]), f1 = mk<T>(X[2], X[3]), f2 = mk<T>(X[4], X[5]),
                 f3 = mk<T>(X[6], X[7]);
    const T da = X[6], db = X[7];
    const T th = T(2) * (norm2(f0) + norm2(f1) + norm2(f2)) + da * da + db * db + (da + db) * (da + db);
    st_stream<T>(Dout + s, f0);
    st_stream<T>(Dout + S + s, f1);
    st_stream<T>(Dout + 2 * S + s, f2);
    st_stream<T>(Dout + 3 * S + s, f3);
    group_sum2<UPDS_THREADS, SITE_BLOCK>((double)tr, (double)th, partials,
                                         blockIdx.x * (UPDS_THREADS / SITE_BLOCK));
}

void update_set_max_lds() {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_update_shared32),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)UPDS_LDS);
}

// reorder 4 fields between natural index order and transform-position order
__global__ void k_reorder(geom g, const double2 *__restrict__ in, long si, double2 *__restrict__ out,
                          long so, int to_natural) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    long r = s;
    const int a0 = (int)(r % g.Lx); r /= g.Lx;
    const int a1 = (int)(r % g.Ly); r /= g.Ly;
    const int a2 = (int)(r % g.Lz);
    const int a3 = (int)(r / g.Lz);
    // s is a position index; its natural (frequency) index:
    const int f0 = fft_freq_of_pos(g.Lx, a0), f1 = fft_freq_of_pos(g.Ly, a1),
              f2 = fft_freq_of_pos(g.Lz, a2), f3 = fft_freq_of_pos(g.Lt, a3);
    const long sn = f0 + (long)g.Lx * (f1 + (long)g.Ly * (f2 + (long)g.Lz * f3));
    for (int f = 0; f < 4; ++f) {
        if (to_natural) out[f * so + sn] = in[f * si + s];
        else out[f * so + s] = in[f * si + sn];
    }
}

__global__ void __launch_bounds__(FIN_BLOCK)
    k_finalize(const double *__restrict__ partials, int nparts, dev_status *__restrict__ status,
               fin_params fp) {
    if (status->done) return;
    double A, B;
    fixed_order_sum<FIN_BLOCK>(partials, nparts, A, B);
    if (threadIdx.x == 0) finalize_state(A, B, status, fp);
}

__global__ void k_status_reset(dev_status *status, int hist_base) {
    dev_status st;
    st.F = 0;
    st.theta = 0;
    st.theta_prev = 0;
    st.theta_min = 0;
    st.n = 0;
    st.done = 0;
    st.code = ST_RUNNING;
    st.rises = 0;
    st.hist_base = hist_base;
    st.since_min = 0;
    *status = st;
}

__global__ void __launch_bounds__(FIN_BLOCK)
    k_measure_finalize(const double *__restrict__ partials, int nparts, double *out2,
                       double normF, double normT) {
    double A, B;
    fixed_order_sum<FIN_BLOCK>(partials, nparts, A, B);
    if (threadIdx.x == 0) {
        out2[0] = A * normF;
        out2[1] = B * normT;
    }
}

__global__ void __launch_bounds__(FIN_BLOCK)
    k_reduce_only(const double *__restrict__ partials, int nparts, double *out2) {
    double A, B;
    fixed_order_sum<FIN_BLOCK>(partials, nparts, A, B);
    if (threadIdx.x == 0) {
        out2[0] = A;
        out2[1] = B;
    }
}

// ---------------------------------------------------------------------------
// mixed precision: accumulated transformation and the hand-over to FP64
// ---------------------------------------------------------------------------

__global__ void k_g_identity(float2 *__restrict__ G, long V, long S) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
#pragma unroll
    for (int k = 0; k < 6; ++k) G[(long)k * S + s] = make_float2(k == 0 || k == 4 ? 1.f : 0.f, 0.f);
}

__device__ __forceinline__ mat3<double> load_G_fp64(const float2 *__restrict__ G, long S, long s) {
    mat3<double> m;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float2 v = G[(long)k * S + s];
        m.e[k / 3][k % 3] = mk<double>(v.x, v.y);
    }
    reunitarise(m);
    return m;
}

// U_mu(x) = G(x) U0_mu(x) G(x+mu)^dagger in FP64, G reunitarised in FP64
template <int LF>
__global__ void __launch_bounds__(SITE_BLOCK)
    k_switch(geom g, const float2 *__restrict__ G, const double2 *__restrict__ U0,
             double2 *__restrict__ L) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const nbr n = neighbours(g, s);
    const mat3<double> g0 = load_G_fp64(G, g.S, s);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const mat3<double> gp = load_G_fp64(G, g.S, n.p[mu]);
        const mat3<double> u = aos_link<double, LF>(U0 + ((long)mu * g.V + s) * 9);
        store_link<double, LF>(L, g.S, mu, s, mul_abcd<product_rows<LF>()>(g0, u, gp));
    }
}

// The hand-over fused with the first FP64 divergence: the links of x as in
// k_switch (stored), the links U_mu(x-mu) formed again from G(x-mu), U0 and
// G(x) exactly as their own site forms them, then Delta(x) and the block
// partials of F and theta, as k_div_reduce would compute them from the stored
// links (the same values in the same order).
template <int LF, class TF>
__global__ void __launch_bounds__(SITE_BLOCK)
    k_switch_div(geom g, const float2 *__restrict__ G, const double2 *__restrict__ U0,
                 double2 *__restrict__ L, vec2_t<TF> *__restrict__ D, double *__restrict__ partials) {
    const long s = block_site(g, blockIdx.x, gridDim.x, threadIdx.x);
    double fs = 0, ts = 0;
    if (s < g.V) {
        const nbr n = neighbours(g, s);
        const mat3<double> g0 = load_G_fp64(G, g.S, s);
        xacc<double> X;
        xacc_zero(X);
        double tr = 0;
        auto aos = [&](int mu, long x) { return aos_link<double, LF>(U0 + ((long)mu * g.V + x) * 9); };
        constexpr int PR = product_rows<LF>();
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const mat3<double> un = mul_abcd<PR>(g0, aos(mu, s), load_G_fp64(G, g.S, n.p[mu]));
            store_link<double, LF>(L, g.S, mu, s, un);
            const mat3<double> u = as_stored<double, LF>(un);  // as loaded back
            tr += retrace(u);
            xacc_add(X, u, -1.0);
            const mat3<double> um =
                as_stored<double, LF>(mul_abcd<PR>(load_G_fp64(G, g.S, n.m[mu]), aos(mu, n.m[mu]), g0));
            xacc_add(X, um, 1.0);
        }
        cpx<double> f0, f1, f2, f3;
        ts = delta_pack(X, f0, f1, f2, f3);
        fs = tr;
        st<TF>(D + s, cvt<TF>(f0));
        st<TF>(D + g.S + s, cvt<TF>(f1));
        st<TF>(D + 2 * g.S + s, cvt<TF>(f2));
        st<TF>(D + 3 * g.S + s, cvt<TF>(f3));
    }
    block_sum2<SITE_BLOCK>(fs, ts, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// gauge-invariant checks and F_U[g]
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(SITE_BLOCK)
    k_plaquette(geom g, const double2 *__restrict__ L, double *__restrict__ partials) {
    const long s = (long)blockIdx.x * SITE_BLOCK + threadIdx.x;
    double acc = 0;
    if (s < g.V) {
        const nbr n = neighbours(g, s);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const mat3<double> umu = load_link<double>(L, g.S, mu, s);
#pragma unroll
            for (int nu = mu + 1; nu < 4; ++nu) {
                const mat3<double> a = load_link<double>(L, g.S, nu, n.p[mu]);   // U_nu(x+mu)
                const mat3<double> b = load_link<double>(L, g.S, mu, n.p[nu]);   // U_mu(x+nu)
                const mat3<double> c = load_link<double>(L, g.S, nu, s);         // U_nu(x)
                // Re Tr[umu a b^+ c^+] = Re Tr[P Q^+] = Re sum_ij P_ij conj(Q_ij),
                // P = umu a, Q = c b
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        cpx<double> p = mk<double>(0, 0), q = mk<double>(0, 0);
                        for (int k = 0; k < 3; ++k) {
                            p = p + cmul(umu.e[i][k], a.e[k][j]);
                            q = q + cmul(c.e[i][k], b.e[k][j]);
                        }
                        acc += p.re * q.re + p.im * q.im;
                    }
            }
        }
    }
    block_sum2<SITE_BLOCK>(acc, 0.0, partials, blockIdx.x);
}

// sum_mu Re Tr[g(x) U_mu(x) g(x+mu)^dagger], g full 3x3 AoS (NULL: identity)
__global__ void __launch_bounds__(SITE_BLOCK)
    k_functional_g(geom g, const double2 *__restrict__ L, const double2 *__restrict__ ga,
                   double *__restrict__ partials) {
    const long s = (long)blockIdx.x * SITE_BLOCK + threadIdx.x;
    double acc = 0;
    if (s < g.V) {
        const nbr n = neighbours(g, s);
        mat3<double> g0;
        for (int k = 0; k < 9; ++k) g0.e[k / 3][k % 3] = mk<double>(ga[s * 9 + k].x, ga[s * 9 + k].y);
        for (int mu = 0; mu < 4; ++mu) {
            mat3<double> gp;
            const long sp = n.p[mu];
            for (int k = 0; k < 9; ++k) gp.e[k / 3][k % 3] = mk<double>(ga[sp * 9 + k].x, ga[sp * 9 + k].y);
            const mat3<double> u = load_link<double>(L, g.S, mu, s);
            // Re Tr[g0 u gp^+] = Re sum_ij (g0 u)_ij conj(gp_ij)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    cpx<double> p = mk<double>(0, 0);
                    for (int k = 0; k < 3; ++k) p = p + cmul(g0.e[i][k], u.e[k][j]);
                    acc += p.re * gp.e[i][j].re + p.im * gp.e[i][j].im;
                }
        }
    }
    block_sum2<SITE_BLOCK>(acc, 0.0, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// differentiation
// ---------------------------------------------------------------------------

// X = i sum_a w_a lambda_a / 2
__device__ __forceinline__ mat3<double> su3_alg(const double *w) {
    const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
    // H = sum_a w_a lambda_a, X = (i/2) H
    cpx<double> H[3][3];
    H[0][0] = mk<double>(w[2] + w[7] * r3, 0);
    H[1][1] = mk<double>(-w[2] + w[7] * r3, 0);
    H[2][2] = mk<double>(-2 * w[7] * r3, 0);
    H[0][1] = mk<double>(w[0], -w[1]);
    H[1][0] = mk<double>(w[0], w[1]);
    H[0][2] = mk<double>(w[3], -w[4]);
    H[2][0] = mk<double>(w[3], w[4]);
    H[1][2] = mk<double>(w[5], -w[6]);
    H[2][1] = mk<double>(w[5], w[6]);
    mat3<double> X;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) X.e[i][j] = mk<double>(-0.5 * H[i][j].im, 0.5 * H[i][j].re);
    return X;
}

__device__ __forceinline__ mat3<double> mat_mul_full(const mat3<double> &a, const mat3<double> &b) {
    mat3<double> r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cpx<double> acc = cmul(a.e[i][0], b.e[0][j]);
            acc = acc + cmul(a.e[i][1], b.e[1][j]);
            acc = acc + cmul(a.e[i][2], b.e[2][j]);
            r.e[i][j] = acc;
        }
    return r;
}

// exp(X) for anti-hermitian X: halve until |X| <= 1/2, Taylor to 24 terms, square back
__device__ mat3<double> expm3(mat3<double> X) {
    double nrm = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) nrm += norm2(X.e[i][j]);
    nrm = sqrt(nrm);
    int sq = 0;
    while (nrm > 0.5 && sq < 60) {
        nrm *= 0.5;
        ++sq;
    }
    const double sc = ldexp(1.0, -sq);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) X.e[i][j] = sc * X.e[i][j];
    mat3<double> E, term;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) E.e[i][j] = term.e[i][j] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
    for (int k = 1; k <= 24; ++k) {
        term = mat_mul_full(term, X);
        const double inv = 1.0 / k;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                term.e[i][j] = inv * term.e[i][j];
                E.e[i][j] = E.e[i][j] + term.e[i][j];
            }
    }
    for (int i = 0; i < sq; ++i) E = mat_mul_full(E, E);
    return E;
}

__global__ void k_expm_sites(const double *__restrict__ w, double2 *__restrict__ out, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ww[8];
    for (int a = 0; a < 8; ++a) ww[a] = w[i * 8 + a];
    const mat3<double> E = expm3(su3_alg(ww));
    for (int k = 0; k < 9; ++k) out[i * 9 + k] = make_double2(E.e[k / 3][k % 3].re, E.e[k / 3][k % 3].im);
}

__device__ __forceinline__ mat3<double> load_full(const double2 *__restrict__ a, long i) {
    mat3<double> m;
    for (int k = 0; k < 9; ++k) m.e[k / 3][k % 3] = mk<double>(a[i * 9 + k].x, a[i * 9 + k].y);
    return m;
}

// links Lout_mu(x) = g(x) Lin_mu(x) g(x+mu)^dagger (g full AoS, unitary)
__global__ void __launch_bounds__(SITE_BLOCK)
    k_rotate_links(geom g, const double2 *__restrict__ Lin, const double2 *__restrict__ ga,
                   double2 *__restrict__ Lout) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const nbr n = neighbours(g, s);
    const mat3<double> g0 = load_full(ga, s);
    for (int mu = 0; mu < 4; ++mu) {
        const mat3<double> gp = load_full(ga, n.p[mu]);
        const mat3<double> u = load_link<double>(Lin, g.S, mu, s);
        store_link<double>(Lout, g.S, mu, s, mul_abcd(g0, u, gp));
    }
}

// Lout_mu(x) = E_mu(x) Lin_mu(x), E full AoS [4][V]
__global__ void k_left_multiply(const double2 *__restrict__ Lin, const double2 *__restrict__ E,
                                double2 *__restrict__ Lout, long V, long S) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = (int)(i / V);
    const long s = i - (long)mu * V;
    const mat3<double> e = load_full(E, i);
    const mat3<double> u = load_link<double>(Lin, S, mu, s);
    mat3<double> r = mat_mul_full(e, u);
    store_link<double>(Lout, S, mu, s, r);
}

// Im Tr[lambda_a W], a = 0..7
__device__ __forceinline__ void im_tr_lambda(const mat3<double> &W, double y[8]) {
    const double r3 = 0.57735026918962576451;
    y[0] = W.e[1][0].im + W.e[0][1].im;
    y[1] = W.e[0][1].re - W.e[1][0].re;
    y[2] = W.e[0][0].im - W.e[1][1].im;
    y[3] = W.e[2][0].im + W.e[0][2].im;
    y[4] = W.e[0][2].re - W.e[2][0].re;
    y[5] = W.e[2][1].im + W.e[1][2].im;
    y[6] = W.e[1][2].re - W.e[2][1].re;
    y[7] = (W.e[0][0].im + W.e[1][1].im - 2 * W.e[2][2].im) * r3;
}

// out = sum_k (A^T)^k v / (k+1)!,  A[b][a] = coefficient of i T^b in [i w.T, i T^a]
//     = -sum_c f_abc w_c  (SU(3) structure constants).
// This is the transpose of the derivative of the exponential map, so for
// g = exp(i w.T): d/dw^a = sum_b S[b][a] (derivative along i T^b g).
__device__ void dexp_transpose_apply(const double *w, const double *v, double *out) {
    double A[8][8];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) A[i][j] = 0;
    const int tri[9][3] = {{0, 1, 2}, {0, 3, 6}, {0, 5, 4}, {1, 3, 5}, {1, 4, 6},
                           {2, 3, 4}, {2, 6, 5}, {3, 4, 7}, {5, 6, 7}};
    const double h3 = 0.86602540378443864676;
    const double fv[9] = {1.0, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, h3, h3};
    for (int t = 0; t < 9; ++t) {
        const int a = tri[t][0], b = tri[t][1], c = tri[t][2];
        const double v0 = fv[t];
        // f_ijk w_k contributes -f_ijk w_k to A[j][i] for every permutation (i,j,k)
        A[b][a] -= v0 * w[c];  // (a,b,c) +
        A[c][b] -= v0 * w[a];  // (b,c,a) +
        A[a][c] -= v0 * w[b];  // (c,a,b) +
        A[a][b] += v0 * w[c];  // (b,a,c) -
        A[c][a] += v0 * w[b];  // (a,c,b) -
        A[b][c] += v0 * w[a];  // (c,b,a) -
    }
    double term[8], acc[8];
    for (int i = 0; i < 8; ++i) term[i] = acc[i] = v[i];
    for (int k = 1; k <= 80; ++k) {
        double nt[8];
        double mx = 0;
        for (int a = 0; a < 8; ++a) {
            double s = 0;
            for (int b = 0; b < 8; ++b) s += A[b][a] * term[b];
            nt[a] = s / (k + 1);
            mx = fmax(mx, fabs(nt[a]));
        }
        double ma = 0;
        for (int a = 0; a < 8; ++a) {
            term[a] = nt[a];
            acc[a] += nt[a];
            ma = fmax(ma, fabs(acc[a]));
        }
        if (mx <= 1e-18 * ma) break;
    }
    for (int a = 0; a < 8; ++a) out[a] = acc[a];
}

// dF/domega from Delta of the transformed links (D64 fields) and omega
__global__ void k_omega_grad(geom g, const double2 *__restrict__ D, const double *__restrict__ om,
                             double *__restrict__ dF, double normF) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const double2 f0 = D[s], f1 = D[g.S + s], f2 = D[2 * g.S + s], f3 = D[3 * g.S + s];
    mat3<double> M;
    M.e[0][0] = mk<double>(0, f3.x);
    M.e[0][1] = mk<double>(f0.x, f0.y);
    M.e[0][2] = mk<double>(f1.x, f1.y);
    M.e[1][0] = mk<double>(-f0.x, f0.y);
    M.e[1][1] = mk<double>(0, f3.y);
    M.e[1][2] = mk<double>(f2.x, f2.y);
    M.e[2][0] = mk<double>(-f1.x, f1.y);
    M.e[2][1] = mk<double>(-f2.x, f2.y);
    M.e[2][2] = mk<double>(0, -(f3.x + f3.y));
    double y[8], G[8], w[8], out[8];
    im_tr_lambda(M, y);
    // G^b = -(i/4) normF Tr[lambda_b Delta] = (normF/4) Im Tr[lambda_b Delta]
    for (int b = 0; b < 8; ++b) G[b] = 0.25 * normF * y[b];
    for (int a = 0; a < 8; ++a) w[a] = om[s * 8 + a];
    dexp_transpose_apply(w, G, out);
    for (int a = 0; a < 8; ++a) dF[s * 8 + a] = out[a];
}

// dtheta/deps^a_mu(x) at links L (already exp(i eps.T) U); eps may be NULL
__global__ void __launch_bounds__(SITE_BLOCK)
    k_theta_grad(geom g, const double2 *__restrict__ L, const double2 *__restrict__ D,
                 const double *__restrict__ eps, double *__restrict__ dth, double normT) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const nbr n = neighbours(g, s);
    auto fieldmat = [&](long q) {
        const double2 f0 = D[q], f1 = D[g.S + q], f2 = D[2 * g.S + q], f3 = D[3 * g.S + q];
        mat3<double> M;
        M.e[0][0] = mk<double>(0, f3.x);
        M.e[0][1] = mk<double>(f0.x, f0.y);
        M.e[0][2] = mk<double>(f1.x, f1.y);
        M.e[1][0] = mk<double>(-f0.x, f0.y);
        M.e[1][1] = mk<double>(0, f3.y);
        M.e[1][2] = mk<double>(f2.x, f2.y);
        M.e[2][0] = mk<double>(-f1.x, f1.y);
        M.e[2][1] = mk<double>(-f2.x, f2.y);
        M.e[2][2] = mk<double>(0, -(f3.x + f3.y));
        return M;
    };
    const mat3<double> d0 = fieldmat(s);
    for (int mu = 0; mu < 4; ++mu) {
        const mat3<double> dp = fieldmat(n.p[mu]);
        mat3<double> Dd;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Dd.e[i][j] = dp.e[i][j] - d0.e[i][j];
        const mat3<double> u = load_link<double>(L, g.S, mu, s);
        mat3<double> ud;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) ud.e[i][j] = conjg(u.e[j][i]);
        const mat3<double> W1 = mat_mul_full(u, Dd), W2 = mat_mul_full(Dd, ud);
        mat3<double> W;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) W.e[i][j] = W1.e[i][j] + W2.e[i][j];
        double y[8], out[8];
        im_tr_lambda(W, y);
        for (int a = 0; a < 8; ++a) y[a] *= normT;
        const long o = ((long)mu * g.V + s) * 8;
        if (eps) {
            double w[8];
            for (int a = 0; a < 8; ++a) w[a] = eps[o + a];
            dexp_transpose_apply(w, y, out);
        } else {
            for (int a = 0; a < 8; ++a) out[a] = y[a];
        }
        for (int a = 0; a < 8; ++a) dth[o + a] = out[a];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <class T>
hipError_t launch_pack_links(const double *Uaos, void *L, const geom &g, hipStream_t st) {
    if (g.nc == 2) return launch_pack_su2<T>(Uaos, L, g, st);
    auto U = reinterpret_cast<const double2 *>(Uaos);
    auto Lp = static_cast<vec2_t<T> *>(L);
    const long V = g.V, S = g.S;
    if (g.lf == 18) k_pack_links<T, 18><<<nblk(4 * V, 256), 256, 0, st>>>(U, Lp, V, S);
    else if (g.lf == 8) k_pack_links<T, 8><<<nblk(4 * V, 256), 256, 0, st>>>(U, Lp, V, S);
    else k_pack_links<T, 12><<<nblk(4 * V, 256), 256, 0, st>>>(U, Lp, V, S);
    return hipGetLastError();
}
template hipError_t launch_pack_links<double>(const double *, void *, const geom &, hipStream_t);
template hipError_t launch_pack_links<float>(const double *, void *, const geom &, hipStream_t);

hipError_t launch_unpack_links(const void *L64, double *Uaos, const geom &g, hipStream_t st) {
    if (g.nc == 2) return launch_unpack_su2(L64, Uaos, g, st);
    auto Lp = static_cast<const double2 *>(L64);
    auto U = reinterpret_cast<double2 *>(Uaos);
    const long V = g.V, S = g.S;
    if (g.lf == 18) k_unpack_links<18><<<nblk(4 * V, 256), 256, 0, st>>>(Lp, U, V, S);
    else if (g.lf == 8) k_unpack_links<8><<<nblk(4 * V, 256), 256, 0, st>>>(Lp, U, V, S);
    else k_unpack_links<12><<<nblk(4 * V, 256), 256, 0, st>>>(Lp, U, V, S);
    return hipGetLastError();
}

// g(x) = exp((alpha/2) L Delta(x)) exactly, once per site, rows 0,1 into GX
// (the update then reads it at x and its neighbours instead of evaluating the
// series nine times per site).
template <class T, class TF>
__global__ void __launch_bounds__(256)
    k_gauge_exp(geom g, const vec2_t<TF> *__restrict__ LD, vec2_t<T> *__restrict__ GX, T c,
                const dev_status *__restrict__ status) {
    if (status->done) return;
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const mat3<T> m = gauge_exp_from_entries<T>(
        cvt<T>(ld<TF>(LD + s)), cvt<T>(ld<TF>(LD + g.S + s)), cvt<T>(ld<TF>(LD + 2 * g.S + s)),
        cvt<T>(ld<TF>(LD + 3 * g.S + s)), c);
#pragma unroll
    for (int k = 0; k < 6; ++k) st<T>(GX + (long)k * g.S + s, m.e[k / 3][k % 3]);
}

// FP32 sweeps of a mixed solve: G(x) <- g(x) G(x), rows 0,1 kept (12 reals),
// from Gold into Gnew (the update then forms G(x) U0 G(x+mu)^dagger at x and
// its neighbours from Gnew; the old G stays readable for those neighbours).
// g and the product are formed and reunitarised in FP64 (accumulate_G).
template <bool EXACT>
__global__ void __launch_bounds__(256)
    k_gauge_acc(geom g, const float2 *__restrict__ LD, const float2 *__restrict__ Gold,
                float2 *__restrict__ Gnew, double c, const dev_status *__restrict__ status) {
    if (status->done) return;
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    accumulate_G<EXACT>(ld<float>(LD + s), ld<float>(LD + g.S + s), ld<float>(LD + 2 * g.S + s),
                        ld<float>(LD + 3 * g.S + s), c, Gold, Gnew, g.S, s);
}

// The Fourier field is FP32 for FP32 sweeps and, when g.ff32 is set, for FP64
// sweeps too; f(tag) runs the body with the field's real type.
template <class T, class Body> hipError_t with_field_type(const geom &g, Body f) {
    if constexpr (std::is_same<T, double>::value) {
        if (g.ff32) return f(float{});
        return f(double{});
    } else {
        return f(float{});
    }
}

template <class T>
hipError_t launch_div_reduce(const geom &g, const void *L, void *D, double *partials,
                             dev_status *status, const fin_params &fp, hipStream_t st) {
    const hipError_t e = with_field_type<T>(g, [&](auto tf) -> hipError_t {
        using TF = decltype(tf);
        auto Lp = static_cast<const vec2_t<T> *>(L);
        auto Dp = static_cast<vec2_t<TF> *>(D);
        if (g.nc == 2) return launch_div_reduce_su2<T, TF>(g, L, D, partials, status, st);
        if (g.lf == 18)
            k_div_reduce<T, TF, 18>
                <<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Lp, Dp, partials, status);
        else if (g.lf == 8)
            k_div_reduce<T, TF, 8>
                <<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Lp, Dp, partials, status);
        else
            k_div_reduce<T, TF, 12>
                <<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Lp, Dp, partials, status);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    if (fp.enabled) k_finalize<<<1, FIN_BLOCK, 0, st>>>(partials, site_blocks(g.V), status, fp);
    return hipGetLastError();
}
template hipError_t launch_div_reduce<double>(const geom &, const void *, void *, double *,
                                              dev_status *, const fin_params &, hipStream_t);
template hipError_t launch_div_reduce<float>(const geom &, const void *, void *, double *,
                                             dev_status *, const fin_params &, hipStream_t);

template <class T>
hipError_t launch_update(const geom &g, const void *Lin, void *Lout, const void *LD, void *Dout,
                         void *G, T c, bool exact, void *GX, double *partials, dev_status *status,
                         const fin_params &fp, hipStream_t st) {
    // G (the accumulated transformation) exists only in the FP32 phase
    constexpr bool ACC = std::is_same<T, float>::value;
    if ((G != nullptr) != ACC) return hipErrorInvalidValue;
    const hipError_t e = with_field_type<T>(g, [&](auto tf) -> hipError_t {
        using TF = decltype(tf);
        if (g.nc == 2)
            return launch_update_su2<T, TF>(g, Lin, Lout, LD, Dout, G, c, exact, partials, status,
                                            st);
        auto LDp = static_cast<const vec2_t<TF> *>(LD);
        if (ACC || exact) {
            if (!GX) return hipErrorInvalidValue;
            // FP32: GX already holds g G (launch_fft_xy_inv_acc / launch_gauge_acc)
            if constexpr (!ACC)
                k_gauge_exp<T, TF><<<nblk(g.V, 256), 256, 0, st>>>(
                    g, LDp, static_cast<vec2_t<T> *>(GX), c, status);
        }
        auto go = [&](auto kernel) {
            kernel<<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(
                g, static_cast<const vec2_t<T> *>(Lin), static_cast<vec2_t<T> *>(Lout), LDp,
                static_cast<const vec2_t<T> *>(GX), static_cast<vec2_t<TF> *>(Dout), c, partials,
                status);
        };
        if constexpr (ACC) {
            // links G U0 G^dagger from the constant copy U0 (Lin), not stored
            if (update_shared_ok(g)) {
                k_update_shared32<<<(unsigned)(g.V / UPDS_THREADS), UPDS_THREADS, UPDS_LDS, st>>>(
                    g, static_cast<const float2 *>(Lin), static_cast<const float2 *>(GX),
                    static_cast<float2 *>(Dout), partials, status);
                return hipGetLastError();
            }
            if (g.lf == 18) go(k_update<T, TF, true, 18, false>);
            else if (g.lf == 8) go(k_update<T, TF, true, 8, false>);
            else go(k_update<T, TF, true, 12, false>);
        } else if (g.lf == 18) {
            if (exact) go(k_update<T, TF, true, 18, true>);
            else go(k_update<T, TF, false, 18, true>);
        } else if (g.lf == 8) {
            if (exact) go(k_update<T, TF, true, 8, true>);
            else go(k_update<T, TF, false, 8, true>);
        } else {
            if (exact) go(k_update<T, TF, true, 12, true>);
            else go(k_update<T, TF, false, 12, true>);
        }
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    if (fp.enabled) k_finalize<<<1, FIN_BLOCK, 0, st>>>(partials, site_blocks(g.V), status, fp);
    return hipGetLastError();
}
hipError_t launch_gauge_acc(const geom &g, const void *LD, const void *Gold, void *Gnew, double c,
                            bool exact, const dev_status *status, hipStream_t st) {
    if (g.nc != 3) return hipErrorInvalidValue;
    auto LDp = static_cast<const float2 *>(LD);
    auto Go = static_cast<const float2 *>(Gold);
    auto Gn = static_cast<float2 *>(Gnew);
    if (exact) k_gauge_acc<true><<<nblk(g.V, 256), 256, 0, st>>>(g, LDp, Go, Gn, c, status);
    else k_gauge_acc<false><<<nblk(g.V, 256), 256, 0, st>>>(g, LDp, Go, Gn, c, status);
    return hipGetLastError();
}

template hipError_t launch_update<double>(const geom &, const void *, void *, const void *, void *,
                                          void *, double, bool, void *, double *, dev_status *,
                                          const fin_params &, hipStream_t);
template hipError_t launch_update<float>(const geom &, const void *, void *, const void *, void *,
                                         void *, float, bool, void *, double *, dev_status *,
                                         const fin_params &, hipStream_t);

hipError_t launch_reorder_fields(const geom &g, const double2 *in, long si, double2 *out, long so,
                                 int to_natural, hipStream_t st) {
    k_reorder<<<nblk(g.V, 256), 256, 0, st>>>(g, in, si, out, so, to_natural);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nparts, dev_status *status,
                           const fin_params &fp, hipStream_t st) {
    k_finalize<<<1, FIN_BLOCK, 0, st>>>(partials, nparts, status, fp);
    return hipGetLastError();
}

hipError_t launch_status_reset(dev_status *status, int hist_base, hipStream_t st) {
    k_status_reset<<<1, 1, 0, st>>>(status, hist_base);
    return hipGetLastError();
}

hipError_t launch_reduce_only(const double *partials, int nparts, double *out2, hipStream_t st) {
    k_reduce_only<<<1, FIN_BLOCK, 0, st>>>(partials, nparts, out2);
    return hipGetLastError();
}

hipError_t launch_measure_aos(const geom &g, const double *Uaos, double *partials, double *out,
                              double normF, double normT, hipStream_t st) {
    const int nb = site_blocks(g.V);
    k_measure_aos<<<nb, SITE_BLOCK, 0, st>>>(g, reinterpret_cast<const double2 *>(Uaos), partials);
    k_measure_finalize<<<1, FIN_BLOCK, 0, st>>>(partials, nb, out, normF, normT);
    return hipGetLastError();
}

hipError_t launch_g_identity(void *G32, const geom &g, hipStream_t st) {
    if (g.nc == 2) return launch_g_identity_su2(G32, g, st);
    k_g_identity<<<nblk(g.V, 256), 256, 0, st>>>(static_cast<float2 *>(G32), g.V, g.S);
    return hipGetLastError();
}

hipError_t launch_switch(const geom &g, const void *G32, const double *U0aos, void *L64,
                         hipStream_t st) {
    if (g.nc == 2) return launch_switch_su2(g, G32, U0aos, L64, st);
    auto Gp = static_cast<const float2 *>(G32);
    auto U0 = reinterpret_cast<const double2 *>(U0aos);
    auto Lp = static_cast<double2 *>(L64);
    if (g.lf == 18) k_switch<18><<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Gp, U0, Lp);
    else if (g.lf == 8) k_switch<8><<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Gp, U0, Lp);
    else k_switch<12><<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Gp, U0, Lp);
    return hipGetLastError();
}

hipError_t launch_switch_div(const geom &g, const void *G32, const double *U0aos, void *L64,
                             void *D, double *partials, dev_status *status, const fin_params &fp,
                             hipStream_t st) {
    if (g.nc != 3) return hipErrorInvalidValue;
    const hipError_t e = with_field_type<double>(g, [&](auto tf) -> hipError_t {
        using TF = decltype(tf);
        auto Gp = static_cast<const float2 *>(G32);
        auto U0 = reinterpret_cast<const double2 *>(U0aos);
        auto Lp = static_cast<double2 *>(L64);
        auto Dp = static_cast<vec2_t<TF> *>(D);
        if (g.lf == 18)
            k_switch_div<18, TF><<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Gp, U0, Lp, Dp, partials);
        else if (g.lf == 8)
            k_switch_div<8, TF><<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Gp, U0, Lp, Dp, partials);
        else
            k_switch_div<12, TF><<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, Gp, U0, Lp, Dp, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    if (fp.enabled) k_finalize<<<1, FIN_BLOCK, 0, st>>>(partials, site_blocks(g.V), status, fp);
    return hipGetLastError();
}

hipError_t launch_field_from_matrix(const double *Maos, void *D64, long V, long S, hipStream_t st) {
    k_field_from_matrix<<<nblk(V, 256), 256, 0, st>>>(reinterpret_cast<const double2 *>(Maos),
                                                      static_cast<double2 *>(D64), V, S);
    return hipGetLastError();
}

hipError_t launch_matrix_from_field(const void *D64, double *Maos, long V, long S, hipStream_t st) {
    k_matrix_from_field<<<nblk(V, 256), 256, 0, st>>>(static_cast<const double2 *>(D64),
                                                      reinterpret_cast<double2 *>(Maos), V, S);
    return hipGetLastError();
}

hipError_t launch_plaquette(const geom &g, const void *L64, double *partials, hipStream_t st) {
    k_plaquette<<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(g, static_cast<const double2 *>(L64),
                                                         partials);
    return hipGetLastError();
}

hipError_t launch_functional_g(const geom &g, const void *L64, const double *gaos,
                               double *partials, hipStream_t st) {
    k_functional_g<<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(
        g, static_cast<const double2 *>(L64), reinterpret_cast<const double2 *>(gaos), partials);
    return hipGetLastError();
}

hipError_t launch_expm_sites(const double *omega, double *gaos, long n, hipStream_t st) {
    k_expm_sites<<<nblk(n, 128), 128, 0, st>>>(omega, reinterpret_cast<double2 *>(gaos), n);
    return hipGetLastError();
}

hipError_t launch_rotate_links(const geom &g, const void *Lin, const double *gaos, void *Lout,
                               hipStream_t st) {
    k_rotate_links<<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(
        g, static_cast<const double2 *>(Lin), reinterpret_cast<const double2 *>(gaos),
        static_cast<double2 *>(Lout));
    return hipGetLastError();
}

hipError_t launch_left_multiply_links(const void *Lin, const double *eaos, void *Lout, long V,
                                      long S, hipStream_t st) {
    k_left_multiply<<<nblk(4 * V, 256), 256, 0, st>>>(static_cast<const double2 *>(Lin),
                                                      reinterpret_cast<const double2 *>(eaos),
                                                      static_cast<double2 *>(Lout), V, S);
    return hipGetLastError();
}

hipError_t launch_omega_grad(const geom &g, const void *D64, const double *omega, double *dF,
                             double normF, hipStream_t st) {
    k_omega_grad<<<nblk(g.V, 128), 128, 0, st>>>(g, static_cast<const double2 *>(D64), omega, dF,
                                                 normF);
    return hipGetLastError();
}

hipError_t launch_theta_grad(const geom &g, const void *L64, const void *D64, const double *eps,
                             double *dth, double normT, hipStream_t st) {
    k_theta_grad<<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(
        g, static_cast<const double2 *>(L64), static_cast<const double2 *>(D64), eps, dth, normT);
    return hipGetLastError();
}

}  // namespace lgf
