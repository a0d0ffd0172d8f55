// SU(2) sweep kernels: the same method with N_c = 2 (the paper's functional
// is written for general N_c).
//
// An SU(2) matrix is [[a, b], [-conj(b), conj(a)]] with |a|^2 + |b|^2 = 1, so
// a working link stores only (a, b) = row 0: 2 complex entries, SoA
// L[(mu*2 + k)*S + s].  Sums and differences of such matrices keep the form,
// so X = sum_mu [U_mu(x-mu) - U_mu(x)] = [[p, q], [-conj(q), conj(p)]] and
// Delta = X - X^dagger = [[2i Im p, 2q], [-2conj(q), -2i Im p]] is already
// traceless.  Its 3 reals travel as 2 complex Fourier fields:
// f0 = Delta01, f1 = Im Delta00 (+ 0i).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "su3.hpp"

namespace lgf {

namespace {

template <class T> struct quat {
    cpx<T> a, b;  // row 0 of [[a, b], [-conj(b), conj(a)]]
};

// (a1,b1)(a2,b2): row 0 of the product
template <class T> LGF_HD quat<T> qmul(const quat<T> &x, const quat<T> &y) {
    return {cmul(x.a, y.a) - cmulc(x.b, y.b), cmul(x.a, y.b) + cmulc(x.b, y.a)};
}
// x y^dagger, y^dagger = (conj(a), -b)
template <class T> LGF_HD quat<T> qmul_dag(const quat<T> &x, const quat<T> &y) {
    return {cmulc(x.a, y.a) + cmulc(x.b, y.b), cmul(x.b, y.a) - cmul(x.a, y.b)};
}

// g = reunit(1 + c M) (first order) or exp(c M) (EXACT) for
// M = [[i alpha, beta], [-conj(beta), -i alpha]], beta = f0, alpha = f1.re.
template <class T, bool EXACT> LGF_HD quat<T> gauge_su2(cpx<T> f0, cpx<T> f1, T c) {
    const T al = c * f1.re;
    const cpx<T> be = c * f0;
    if constexpr (EXACT) {
        // c M = i v.sigma with |v|^2 = al^2 + |be|^2: exp = cos|v| + (sin|v|/|v|) c M
        const T w2 = al * al + norm2(be);
        T cw, sw;
        if (w2 < T(1e-6)) {
            cw = T(1) - w2 * (T(0.5) - w2 * T(1.0 / 24.0));
            sw = T(1) - w2 * (T(1.0 / 6.0) - w2 * T(1.0 / 120.0));
        } else {
            const T w = sqrt(w2);
            T sn;
            if constexpr (std::is_same<T, float>::value) sincosf(w, &sn, &cw);
            else sincos(w, &sn, &cw);
            sw = sn / w;
        }
        return {mk<T>(cw, sw * al), sw * be};
    } else {
        const T r = rsqrt_nr(T(1) + al * al + norm2(be));
        return {mk<T>(r, r * al), r * be};
    }
}

template <class T> LGF_HD quat<T> load_q(const vec2_t<T> *__restrict__ L, long S, int mu, long s) {
    const vec2_t<T> *p = L + (long)mu * 2 * S + s;
    return {ld<T>(p), ld<T>(p + S)};
}

template <class T> LGF_HD void store_q(vec2_t<T> *__restrict__ L, long S, int mu, long s,
                                       const quat<T> &u) {
    vec2_t<T> *p = L + (long)mu * 2 * S + s;
    st_stream<T>(p, u.a);
    st_stream<T>(p + S, u.b);
}

// Delta fields (real type TF) and Tr[Delta Delta^dagger] from the
// accumulated (p, q)
template <class T, class TF>
LGF_HD T delta_su2(cpx<T> p, cpx<T> q, vec2_t<TF> *__restrict__ D, long S, long s) {
    st_stream<TF>(D + s, cvt<TF>(T(2) * q));
    st_stream<TF>(D + S + s, cvt<TF>(mk<T>(T(2) * p.im, 0)));
    return T(8) * (p.im * p.im + norm2(q));
}

}  // namespace

template <class T>
__global__ void __launch_bounds__(256) k_pack_su2(const double2 *__restrict__ U,
                                                  vec2_t<T> *__restrict__ L, long V, long S) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = (int)(i / V);
    const long s = i - (long)mu * V;
    const double2 *u = U + i * 4;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        vec2_t<T> w;
        w.x = (T)u[k].x;
        w.y = (T)u[k].y;
        L[((long)mu * 2 + k) * S + s] = w;
    }
}

__global__ void __launch_bounds__(256) k_unpack_su2(const double2 *__restrict__ L,
                                                    double2 *__restrict__ U, long V, long S) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = (int)(i / V);
    const long s = i - (long)mu * V;
    const double2 a = L[((long)mu * 2) * S + s], b = L[((long)mu * 2 + 1) * S + s];
    double2 *u = U + i * 4;
    u[0] = a;
    u[1] = b;
    u[2] = make_double2(-b.x, b.y);
    u[3] = make_double2(a.x, -a.y);
}

template <class T, class TF>
__global__ void __launch_bounds__(SITE_BLOCK)
    k_div_reduce_su2(geom g, const vec2_t<T> *__restrict__ L, vec2_t<TF> *__restrict__ D,
                     double *__restrict__ partials, const dev_status *__restrict__ status) {
    if (status->done) return;
    const long s = block_site(g, blockIdx.x, gridDim.x, threadIdx.x);
    double fs = 0, ts = 0;
    if (s < g.V) {
        const nbr n = neighbours(g, s);
        cpx<T> p = mk<T>(0, 0), q = mk<T>(0, 0);
        T tr = 0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const quat<T> u = load_q<T>(L, g.S, mu, s), um = load_q<T>(L, g.S, mu, n.m[mu]);
            tr += T(2) * u.a.re;
            p = p + (um.a - u.a);
            q = q + (um.b - u.b);
        }
        ts = (double)delta_su2<T, TF>(p, q, D, g.S, s);
        fs = (double)tr;
    }
    block_sum2<SITE_BLOCK>(fs, ts, partials, blockIdx.x);
}

// U_mu(x) <- g(x) U_mu(x) g(x+mu)^dagger, fused with the next Delta (which needs
// the new U_mu(x-mu) = g(x-mu) U_mu(x-mu) g(x)^dagger) and the F/theta partials.
// ACC_G (the FP32 phase of a mixed solve): also G(x) <- g(x) G(x), G stored as
// its row 0 like the links, formed and normalised in FP64.
template <class T, class TF, bool EXACT, bool ACC_G>
__global__ void __launch_bounds__(SITE_BLOCK)
    k_update_su2(geom g, const vec2_t<T> *__restrict__ Lin, vec2_t<T> *__restrict__ Lout,
                 const vec2_t<TF> *__restrict__ LD, vec2_t<TF> *__restrict__ Dout,
                 vec2_t<T> *__restrict__ G, T c, double *__restrict__ partials,
                 const dev_status *__restrict__ status) {
    if (status->done) return;
    const long s = block_site(g, blockIdx.x, gridDim.x, threadIdx.x);
    double fs = 0, ts = 0;
    if (s < g.V) {
        const nbr n = neighbours(g, s);
        auto gauge_at = [&](long x) {
            return gauge_su2<T, EXACT>(cvt<T>(ld<TF>(LD + x)), cvt<T>(ld<TF>(LD + g.S + x)), c);
        };
        const quat<T> g0 = gauge_at(s);
        cpx<T> p = mk<T>(0, 0), q = mk<T>(0, 0);
        T tr = 0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const quat<T> gp = gauge_at(n.p[mu]), gm = gauge_at(n.m[mu]);
            const quat<T> u = load_q<T>(Lin, g.S, mu, s), um = load_q<T>(Lin, g.S, mu, n.m[mu]);
            const quat<T> un = qmul_dag(qmul(g0, u), gp);    // g(x) U_mu(x) g(x+mu)^+
            const quat<T> umn = qmul_dag(qmul(gm, um), g0);  // g(x-mu) U_mu(x-mu) g(x)^+
            store_q<T>(Lout, g.S, mu, s, un);
            tr += T(2) * un.a.re;
            p = p + (umn.a - un.a);
            q = q + (umn.b - un.b);
        }
        ts = (double)delta_su2<T, TF>(p, q, Dout, g.S, s);
        fs = (double)tr;
        if constexpr (ACC_G) {
            // g formed, multiplied into G and the product normalised in FP64;
            // only the stored row of G is rounded to FP32
            const quat<double> g64 = gauge_su2<double, EXACT>(
                cvt<double>(ld<TF>(LD + s)), cvt<double>(ld<TF>(LD + g.S + s)), (double)c);
            const quat<double> Gn = qmul(
                g64, quat<double>{cvt<double>(ld<T>(G + s)), cvt<double>(ld<T>(G + g.S + s))});
            const double r = rsqrt_nr(norm2(Gn.a) + norm2(Gn.b));
            st<T>(G + s, cvt<T>(r * Gn.a));
            st<T>(G + g.S + s, cvt<T>(r * Gn.b));
        }
    }
    block_sum2<SITE_BLOCK>(fs, ts, partials, blockIdx.x);
}

// mixed precision: G = 1, and the hand-over U = G U0 G(x+mu)^dagger in FP64
// with G normalised in FP64
__global__ void k_g_identity_su2(float2 *__restrict__ G, long V, long S) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    G[s] = make_float2(1.f, 0.f);
    G[S + s] = make_float2(0.f, 0.f);
}

__device__ __forceinline__ quat<double> load_G_su2(const float2 *__restrict__ G, long S, long s) {
    const float2 a = G[s], b = G[S + s];
    const quat<double> q{mk<double>(a.x, a.y), mk<double>(b.x, b.y)};
    const double r = rsqrt_nr(norm2(q.a) + norm2(q.b));
    return {r * q.a, r * q.b};
}

__global__ void __launch_bounds__(SITE_BLOCK)
    k_switch_su2(geom g, const float2 *__restrict__ G, const double2 *__restrict__ U0,
                 double2 *__restrict__ L) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    const nbr n = neighbours(g, s);
    const quat<double> g0 = load_G_su2(G, g.S, s);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const quat<double> gp = load_G_su2(G, g.S, n.p[mu]);
        const double2 *p = U0 + ((long)mu * g.V + s) * 4;
        const quat<double> u{mk<double>(p[0].x, p[0].y), mk<double>(p[1].x, p[1].y)};
        store_q<double>(L, g.S, mu, s, qmul_dag(qmul(g0, u), gp));
    }
}

static inline unsigned nblk2(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <class T>
hipError_t launch_pack_su2(const double *Uaos, void *L, const geom &g, hipStream_t st) {
    k_pack_su2<T><<<nblk2(4 * g.V, 256), 256, 0, st>>>(reinterpret_cast<const double2 *>(Uaos),
                                                       static_cast<vec2_t<T> *>(L), g.V, g.S);
    return hipGetLastError();
}
template hipError_t launch_pack_su2<double>(const double *, void *, const geom &, hipStream_t);
template hipError_t launch_pack_su2<float>(const double *, void *, const geom &, hipStream_t);

hipError_t launch_unpack_su2(const void *L64, double *Uaos, const geom &g, hipStream_t st) {
    k_unpack_su2<<<nblk2(4 * g.V, 256), 256, 0, st>>>(static_cast<const double2 *>(L64),
                                                      reinterpret_cast<double2 *>(Uaos), g.V, g.S);
    return hipGetLastError();
}

template <class T, class TF>
hipError_t launch_div_reduce_su2(const geom &g, const void *L, void *D, double *partials,
                                 dev_status *status, hipStream_t st) {
    k_div_reduce_su2<T, TF><<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(
        g, static_cast<const vec2_t<T> *>(L), static_cast<vec2_t<TF> *>(D), partials, status);
    return hipGetLastError();
}
template hipError_t launch_div_reduce_su2<double, double>(const geom &, const void *, void *,
                                                          double *, dev_status *, hipStream_t);
template hipError_t launch_div_reduce_su2<double, float>(const geom &, const void *, void *,
                                                         double *, dev_status *, hipStream_t);
template hipError_t launch_div_reduce_su2<float, float>(const geom &, const void *, void *,
                                                        double *, dev_status *, hipStream_t);

template <class T, class TF>
hipError_t launch_update_su2(const geom &g, const void *Lin, void *Lout, const void *LD,
                             void *Dout, void *G, T c, bool exact, double *partials,
                             dev_status *status, hipStream_t st) {
    auto go = [&](auto kernel) {
        kernel<<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(
            g, static_cast<const vec2_t<T> *>(Lin), static_cast<vec2_t<T> *>(Lout),
            static_cast<const vec2_t<TF> *>(LD), static_cast<vec2_t<TF> *>(Dout),
            static_cast<vec2_t<T> *>(G), c, partials, status);
    };
    // G (the accumulated transformation) exists only in the FP32 phase
    constexpr bool ACC = std::is_same<T, float>::value;
    if ((G != nullptr) != ACC) return hipErrorInvalidValue;
    if (exact) go(k_update_su2<T, TF, true, ACC>);
    else go(k_update_su2<T, TF, false, ACC>);
    return hipGetLastError();
}
template hipError_t launch_update_su2<double, double>(const geom &, const void *, void *,
                                                      const void *, void *, void *, double, bool,
                                                      double *, dev_status *, hipStream_t);
template hipError_t launch_update_su2<double, float>(const geom &, const void *, void *,
                                                     const void *, void *, void *, double, bool,
                                                     double *, dev_status *, hipStream_t);
template hipError_t launch_update_su2<float, float>(const geom &, const void *, void *,
                                                    const void *, void *, void *, float, bool,
                                                    double *, dev_status *, hipStream_t);

hipError_t launch_g_identity_su2(void *G32, const geom &g, hipStream_t st) {
    k_g_identity_su2<<<nblk2(g.V, 256), 256, 0, st>>>(static_cast<float2 *>(G32), g.V, g.S);
    return hipGetLastError();
}

hipError_t launch_switch_su2(const geom &g, const void *G32, const double *U0aos, void *L64,
                             hipStream_t st) {
    k_switch_su2<<<site_blocks(g.V), SITE_BLOCK, 0, st>>>(
        g, static_cast<const float2 *>(G32), reinterpret_cast<const double2 *>(U0aos),
        static_cast<double2 *>(L64));
    return hipGetLastError();
}

}  // namespace lgf
