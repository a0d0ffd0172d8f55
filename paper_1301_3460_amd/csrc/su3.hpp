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

// Rows 0,1 of A * B * C^dagger, then row 2 rebuilt (the result is SU(3)
// when A, B, C are).
template <class T> LGF_HD mat3<T> mul_abcd(const mat3<T> &A, const mat3<T> &B, const mat3<T> &C) {
    mat3<T> r;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
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
    rebuild_row2(r);
    return r;
}

// ------------------------------------------------------------------------
// Storage layouts
//   links SoA-12:  L[(mu*6 + k)*S + s], k = 3*row + col, row in {0,1}
//   Fourier field: D[f*S + s], f = 0..3 holding the independent entries of
//                  an anti-hermitian traceless matrix:
//                  f0 = M01, f1 = M02, f2 = M12,
//                  f3 = (Im M00) + i (Im M11)
// ------------------------------------------------------------------------

template <class T>
LGF_HD mat3<T> load_link(const vec2_t<T> *__restrict__ L, long S, int mu, long s) {
    mat3<T> m;
    const vec2_t<T> *p = L + (long)mu * 6 * S + s;
#pragma unroll
    for (int k = 0; k < 6; ++k) m.e[k / 3][k % 3] = ld<T>(p + (long)k * S);
    rebuild_row2(m);
    return m;
}

template <class T>
LGF_HD void store_link(vec2_t<T> *__restrict__ L, long S, int mu, long s, const mat3<T> &m) {
    vec2_t<T> *p = L + (long)mu * 6 * S + s;
#pragma unroll
    for (int k = 0; k < 6; ++k) st<T>(p + (long)k * S, m.e[k / 3][k % 3]);
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
