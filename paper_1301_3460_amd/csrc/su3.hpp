// SU(3) arithmetic for the gauge-fixing kernels, templated on the real type.
//
// Links are stored as 12 reals (rows 0 and 1 of the matrix); row 2 of an
// SU(3) matrix is conj(row0 x row1), so nothing is lost.  Matrices in this
// file are small register arrays; every function is force-inlined.
#pragma once
#include <hip/hip_runtime.h>

namespace lgf {

template <class T> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };
template <class T> using vec2_t = typename vec2<T>::type;

template <class T> struct cpx {
    T re, im;
};

#define LGF_HD __device__ __forceinline__

template <class T> LGF_HD cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <class T> LGF_HD cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> LGF_HD cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> LGF_HD cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
// Complex products are written as explicit fused multiply-add chains: the
// rounding is then fixed by the source (not by the compiler's contraction
// choices), and a multiply-accumulate costs four FMAs.
template <class T> LGF_HD cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// a * conj(b)
template <class T> LGF_HD cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return {fma(a.re, b.re, a.im * b.im), fma(a.im, b.re, -a.re * b.im)};
}
// acc + a * b
template <class T> LGF_HD cpx<T> cmac(cpx<T> acc, cpx<T> a, cpx<T> b) {
    return {fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}
// acc + a * conj(b)
template <class T> LGF_HD cpx<T> cmacc(cpx<T> acc, cpx<T> a, cpx<T> b) {
    return {fma(a.re, b.re, fma(a.im, b.im, acc.re)), fma(a.im, b.re, fma(-a.re, b.im, acc.im))};
}
// acc - a * b
template <class T> LGF_HD cpx<T> cmsub(cpx<T> acc, cpx<T> a, cpx<T> b) {
    return {fma(-a.re, b.re, fma(a.im, b.im, acc.re)), fma(-a.re, b.im, fma(-a.im, b.re, acc.im))};
}
template <class T> LGF_HD cpx<T> conjg(cpx<T> a) { return {a.re, -a.im}; }
template <class T> LGF_HD T norm2(cpx<T> a) { return a.re * a.re + a.im * a.im; }

// a complex value in another precision (the Fourier field of FP64 sweeps may
// be held in FP32)
template <class U, class T> LGF_HD cpx<U> cvt(cpx<T> a) { return {(U)a.re, (U)a.im}; }

template <class T> LGF_HD cpx<T> ld(const vec2_t<T> *p) {
    vec2_t<T> v = *p;
    return {v.x, v.y};
}
template <class T> LGF_HD void st(vec2_t<T> *p, cpx<T> a) {
    vec2_t<T> v;
    v.x = a.re;
    v.y = a.im;
    *p = v;
}

// Streaming store: written once and not read again by this kernel, so it is
// marked non-temporal and does not displace lines that neighbouring blocks
// are still going to read.
template <class T> LGF_HD void st_stream(vec2_t<T> *p, cpx<T> a) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = {a.re, a.im};
    __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
}

// 3x3 complex matrix, row-major.
template <class T> struct mat3 {
    cpx<T> e[3][3];
};

// row 2 = conj(row0 x row1)
template <class T> LGF_HD void rebuild_row2(mat3<T> &m) {
    m.e[2][0] = conjg(cmsub(cmul(m.e[0][1], m.e[1][2]), m.e[0][2], m.e[1][1]));
    m.e[2][1] = conjg(cmsub(cmul(m.e[0][2], m.e[1][0]), m.e[0][0], m.e[1][2]));
    m.e[2][2] = conjg(cmsub(cmul(m.e[0][0], m.e[1][1]), m.e[0][1], m.e[1][0]));
}

// 1/sqrt(x): hardware estimate refined by Newton steps y <- y + y(1 - x y^2)/2
// (two in FP64, one in FP32), to about 1 ulp.
LGF_HD double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}
LGF_HD float rsqrt_nr(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    const float e = fmaf(-x * y, y, 1.0f);
    return fmaf(0.5f * y, e, y);
}

// Gram-Schmidt on rows 0,1 (in place), then rebuild row 2.
template <class T> LGF_HD void reunitarise(mat3<T> &m) {
    T n0 = norm2(m.e[0][0]) + norm2(m.e[0][1]) + norm2(m.e[0][2]);
    T r0 = rsqrt_nr(n0);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[0][j] = r0 * m.e[0][j];
    // <row0, row1> = sum conj(row0_j) row1_j
    cpx<T> ip = cmulc(m.e[1][0], m.e[0][0]);
    ip = cmacc(ip, m.e[1][1], m.e[0][1]);
    ip = cmacc(ip, m.e[1][2], m.e[0][2]);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[1][j] = cmsub(m.e[1][j], ip, m.e[0][j]);
    T n1 = norm2(m.e[1][0]) + norm2(m.e[1][1]) + norm2(m.e[1][2]);
    T r1 = rsqrt_nr(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[1][j] = r1 * m.e[1][j];
    rebuild_row2(m);
}

// A * B * C^dagger.  ROWS = 2: rows 0,1 by products, row 2 rebuilt (the
// result is SU(3) when A, B, C are); ROWS = 3: all three rows by products.
template <int ROWS = 2, class T>
LGF_HD mat3<T> mul_abcd(const mat3<T> &A, const mat3<T> &B, const mat3<T> &C) {
    mat3<T> r;
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
        cpx<T> ab[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cpx<T> acc = cmul(A.e[i][0], B.e[0][k]);
            acc = cmac(acc, A.e[i][1], B.e[1][k]);
            ab[k] = cmac(acc, A.e[i][2], B.e[2][k]);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<T> acc = cmulc(ab[0], C.e[j][0]);
            acc = cmacc(acc, ab[1], C.e[j][1]);
            r.e[i][j] = cmacc(acc, ab[2], C.e[j][2]);
        }
    }
    if constexpr (ROWS == 2) rebuild_row2(r);
    return r;
}

// ------------------------------------------------------------------------
// Storage layouts
//   links SoA:     L[(mu*3*NR + k)*S + s], k = 3*row + col for the NR stored
//                  rows: NR = 2 is the 12-real form (rows 0,1; row 2 rebuilt
//                  as conj(row0 x row1)), NR = 3 the 18-real form (no rebuild)
//   Fourier field: D[f*S + s], f = 0..3 holding the independent entries of
//                  an anti-hermitian traceless matrix:
//                  f0 = M01, f1 = M02, f2 = M12,
//                  f3 = (Im M00) + i (Im M11)
// ------------------------------------------------------------------------

template <class T, int NR = 2>
LGF_HD mat3<T> load_link(const vec2_t<T> *__restrict__ L, long S, int mu, long s) {
    mat3<T> m;
    const vec2_t<T> *p = L + (long)mu * 3 * NR * S + s;
#pragma unroll
    for (int k = 0; k < 3 * NR; ++k) m.e[k / 3][k % 3] = ld<T>(p + (long)k * S);
    if constexpr (NR == 2) rebuild_row2(m);
    return m;
}

template <class T, int NR = 2>
LGF_HD void store_link(vec2_t<T> *__restrict__ L, long S, int mu, long s, const mat3<T> &m) {
    vec2_t<T> *p = L + (long)mu * 3 * NR * S + s;
#pragma unroll
    for (int k = 0; k < 3 * NR; ++k) st_stream<T>(p + (long)k * S, m.e[k / 3][k % 3]);
}

// g = reunit(1 + c * M) for the anti-hermitian traceless M whose 4 Fourier-
// field entries are f (c = alpha/2).  Only rows 0,1 of 1 + cM enter.
template <class T>
LGF_HD mat3<T> gauge_from_entries(cpx<T> f0, cpx<T> f1, cpx<T> f2, cpx<T> f3, T c) {
    mat3<T> g;
    g.e[0][0] = mk<T>(1, c * f3.re);
    g.e[0][1] = c * f0;
    g.e[0][2] = c * f1;
    g.e[1][0] = mk<T>(-c * f0.re, c * f0.im);  // c * (-conj(M01))
    g.e[1][1] = mk<T>(1, c * f3.im);
    g.e[1][2] = c * f2;
    reunitarise(g);
    return g;
}

// g = exp(c * M) exactly, for the same M.  With Q = -i c M (hermitian,
// traceless) the Cayley-Hamilton theorem gives Q^3 = c1 Q + c0 with
// c1 = Tr(Q^2)/2 and c0 = det Q, so every power of Q, and hence exp(iQ), is a
// combination f0 + f1 Q + f2 Q^2.  The f_j are summed from the exponential
// series with the powers reduced by that recurrence (Q^k = a + b Q + d Q^2,
// Q^(k+1) = c0 d + (a + c1 d) Q + b Q^2), after scaling Q by 2^-s so that its
// Frobenius norm is at most 1/2 (16 terms then leave an error below 1e-18);
// s squarings in the same three-term algebra undo the scaling.  No matrix
// products until the end, no transcendental functions.
template <class T>
LGF_HD mat3<T> gauge_exp_from_entries(cpx<T> f0, cpx<T> f1, cpx<T> f2, cpx<T> f3, T c) {
    // Q = -i c M: diagonal c (a, b, -(a+b)); Q01 = -i c f0, Q02 = -i c f1, Q12 = -i c f2
    const T q0 = c * f3.re, q1 = c * f3.im, q2 = -(q0 + q1);
    const cpx<T> Q01 = mk<T>(c * f0.im, -c * f0.re), Q02 = mk<T>(c * f1.im, -c * f1.re),
                 Q12 = mk<T>(c * f2.im, -c * f2.re);
    const T n01 = norm2(Q01), n02 = norm2(Q02), n12 = norm2(Q12);
    const T c1 = T(0.5) * (q0 * q0 + q1 * q1 + q2 * q2) + n01 + n02 + n12;
    // det Q = q0 q1 q2 + 2 Re(Q01 Q12 Q20) - q0 |Q12|^2 - q1 |Q02|^2 - q2 |Q01|^2
    const cpx<T> t = cmulc(cmul(Q01, Q12), Q02);
    const T c0 = q0 * q1 * q2 + T(2) * t.re - q0 * n12 - q1 * n02 - q2 * n01;
    // scaling: |Q|_F^2 = 2 c1 <= 1/4 (bounded loop: a non-finite c1 leaves it)
    int sq = 0;
    T r2 = T(2) * c1;
    while (sq < 64 && r2 > T(0.25)) {
        r2 *= T(0.25);
        ++sq;
    }
    T sc = T(1);
    for (int i = 0; i < sq; ++i) sc *= T(0.5);
    T c1s = c1 * sc * sc, c0s = c0 * sc * sc * sc;
    // series: sum_k i^k/k! (a_k, b_k, d_k)
    cpx<T> F0 = mk<T>(0, 0), F1 = mk<T>(0, 0), F2 = mk<T>(0, 0), fac = mk<T>(1, 0);
    T a = 1, b = 0, d = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        F0 = F0 + a * fac;
        F1 = F1 + b * fac;
        F2 = F2 + d * fac;
        const T an = c0s * d, bn = fma(c1s, d, a);
        d = b;
        a = an;
        b = bn;
        fac = (T(1) / T(k + 1)) * mk<T>(-fac.im, fac.re);  // times i/(k+1)
    }
    // squaring: (F0 + F1 P + F2 P^2)^2 reduced with P^3 = c1s P + c0s, then P -> 2P
    for (int i = 0; i < sq; ++i) {
        const cpx<T> f12 = cmul(F1, F2), f22 = cmul(F2, F2);
        const cpx<T> g0 = cmac(c0s * (T(2) * f12), F0, F0);
        const cpx<T> g1 = cmac(c1s * (T(2) * f12) + c0s * f22, T(2) * F0, F1);
        const cpx<T> g2 = cmac(cmac(c1s * f22, F1, F1), T(2) * F0, F2);
        F0 = g0;
        F1 = T(0.5) * g1;
        F2 = T(0.25) * g2;
        c1s *= T(4);
        c0s *= T(8);
    }
    // rows 0, 1 of f0 + f1 Q + f2 Q^2
    cpx<T> Q[3][3];
    Q[0][0] = mk<T>(q0, 0);
    Q[1][1] = mk<T>(q1, 0);
    Q[2][2] = mk<T>(q2, 0);
    Q[0][1] = Q01;
    Q[0][2] = Q02;
    Q[1][2] = Q12;
    Q[1][0] = conjg(Q01);
    Q[2][0] = conjg(Q02);
    Q[2][1] = conjg(Q12);
    mat3<T> g;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<T> q2ij = cmul(Q[i][0], Q[0][j]);
            q2ij = cmac(q2ij, Q[i][1], Q[1][j]);
            q2ij = cmac(q2ij, Q[i][2], Q[2][j]);
            cpx<T> e = cmac(cmul(F1, Q[i][j]), F2, q2ij);
            if (i == j) e = e + F0;
            g.e[i][j] = e;
        }
    rebuild_row2(g);
    return g;
}

// One step of the accumulated transformation of the FP32 sweeps of a mixed
// solve, G(x) <- g(x) G(x), in FP64: g is formed from the FP32 entries of
// L Delta and made unitary in FP64 (first-order step, Gram-Schmidt) or
// exponentiated in FP64 (exact step); the product with the stored rows 0,1 of
// G (row 2 rebuilt) is reunitarised in FP64, so G stays on SU(3) to FP32
// rounding sweep after sweep; only rows 0,1 of the result are rounded to FP32.
template <bool EXACT>
LGF_HD void accumulate_G(cpx<float> f0, cpx<float> f1, cpx<float> f2, cpx<float> f3, double c,
                         const float2 *__restrict__ Gold, float2 *__restrict__ Gnew, long S,
                         long s) {
    const cpx<double> e0 = cvt<double>(f0), e1 = cvt<double>(f1), e2 = cvt<double>(f2),
                      e3 = cvt<double>(f3);
    mat3<double> gx;
    if constexpr (EXACT) gx = gauge_exp_from_entries<double>(e0, e1, e2, e3, c);
    else gx = gauge_from_entries<double>(e0, e1, e2, e3, c);
    mat3<double> G0;
#pragma unroll
    for (int k = 0; k < 6; ++k) G0.e[k / 3][k % 3] = cvt<double>(ld<float>(Gold + (long)k * S + s));
    rebuild_row2(G0);
    mat3<double> Gn;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cpx<double> acc = cmul(gx.e[r][0], G0.e[0][j]);
            acc = cmac(acc, gx.e[r][1], G0.e[1][j]);
            Gn.e[r][j] = cmac(acc, gx.e[r][2], G0.e[2][j]);
        }
    reunitarise(Gn);
#pragma unroll
    for (int k = 0; k < 6; ++k) st<float>(Gnew + (long)k * S + s, cvt<float>(Gn.e[k / 3][k % 3]));
}

// The same from a Fourier field at site s.
template <class T>
LGF_HD mat3<T> gauge_from_field(const vec2_t<T> *__restrict__ D, long S, long s, T c) {
    return gauge_from_entries<T>(ld<T>(D + s), ld<T>(D + S + s), ld<T>(D + 2 * S + s),
                                 ld<T>(D + 3 * S + s), c);
}

// Accumulator of X = sum_mu [U_mu(x-mu) - U_mu(x)] restricted to what the
// anti-hermitian traceless projection needs.
template <class T> struct xacc {
    cpx<T> x01, x10, x02, x20, x12, x21;
    T i00, i11, i22;
};

template <class T> LGF_HD void xacc_zero(xacc<T> &a) {
    a.x01 = a.x10 = a.x02 = a.x20 = a.x12 = a.x21 = mk<T>(0, 0);
    a.i00 = a.i11 = a.i22 = T(0);
}

// a += sgn * m
template <class T> LGF_HD void xacc_add(xacc<T> &a, const mat3<T> &m, T sgn) {
    a.x01 = a.x01 + sgn * m.e[0][1];
    a.x10 = a.x10 + sgn * m.e[1][0];
    a.x02 = a.x02 + sgn * m.e[0][2];
    a.x20 = a.x20 + sgn * m.e[2][0];
    a.x12 = a.x12 + sgn * m.e[1][2];
    a.x21 = a.x21 + sgn * m.e[2][1];
    a.i00 += sgn * m.e[0][0].im;
    a.i11 += sgn * m.e[1][1].im;
    a.i22 += sgn * m.e[2][2].im;
}

// Delta = (X - X^dagger) - Tr/3, packed into the 4 Fourier-field entries;
// returns Tr[Delta Delta^dagger].
template <class T>
LGF_HD T delta_pack(const xacc<T> &a, cpx<T> &f0, cpx<T> &f1, cpx<T> &f2, cpx<T> &f3) {
    f0 = a.x01 - conjg(a.x10);
    f1 = a.x02 - conjg(a.x20);
    f2 = a.x12 - conjg(a.x21);
    T d0 = T(2) * a.i00, d1 = T(2) * a.i11, d2 = T(2) * a.i22;
    T tr = (d0 + d1 + d2) * T(1.0 / 3.0);
    T da = d0 - tr, db = d1 - tr;
    f3 = mk<T>(da, db);
    return T(2) * (norm2(f0) + norm2(f1) + norm2(f2)) + da * da + db * db + (da + db) * (da + db);
}

template <class T> LGF_HD T retrace(const mat3<T> &m) {
    return m.e[0][0].re + m.e[1][1].re + m.e[2][2].re;
}

}  // namespace lgf
