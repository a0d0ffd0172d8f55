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

// 1/x from the hardware estimate refined by Newton steps (to about 1 ulp).
LGF_HD double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
LGF_HD float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
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
// Minimal 8-real link storage
//
// An SU(3) matrix has 8 real degrees of freedom, but no single set of 8
// matrix coordinates covers the group without a singular set (the usual
// form, U01, U02, U10 and the phases of U00 and U20, divides by 1 - |U00|^2
// and loses the lower block entirely on diagonal links).  Here every link is
// first brought to a well-conditioned frame V = R U P: P permutes the columns
// so that row 0 reads (smallest, middle, largest modulus) and R swaps rows 1
// and 2 when that makes |V20| >= |V10|.  Then |V00|^2 <= 1/3, |V02|^2 >= 1/3
// and |V20|^2 >= 1/3, and the stored reals are
//     V00 (2), V01 (2), V10 (2), tan(phi/4) of the phases of V02 and V20 (2),
// with the permutation (3 columns x parity, 2 bits) and the row swap (1 bit)
// in the two lowest mantissa bits of Re V01 and Im V01.  Decoding derives
// |V02| and |V20| from the unit norms of row 0 and column 0 (no cancellation:
// both are at least 1/3), the remaining 2x2 block from the cofactor identity
// of a unitary matrix of determinant d = det R det P = +-1,
//     conj(V_ij) = C_ij / d,
// which divides only by 1 - |V00|^2 >= 2/3, and undoes R and P.  The phase
// codes are rational in tan(phi/4) (no trigonometric functions), and every
// step is well conditioned, so a round trip changes a link by about 1e-15 in
// FP64.  The tag bits perturb Re V01 and Im V01 by at most 3 ulp.
// ------------------------------------------------------------------------

LGF_HD double with_tag(double v, int b) {
    return __longlong_as_double((__double_as_longlong(v) & ~3LL) | (long long)b);
}
LGF_HD float with_tag(float v, int b) { return __int_as_float((__float_as_int(v) & ~3) | b); }
LGF_HD int tag_of(double v) { return (int)(__double_as_longlong(v) & 3); }
LGF_HD int tag_of(float v) { return __float_as_int(v) & 3; }
LGF_HD double untag(double v) { return __longlong_as_double(__double_as_longlong(v) & ~3LL); }
LGF_HD float untag(float v) { return __int_as_float(__float_as_int(v) & ~3); }

// tan(phi/4) of z = |z| e^{i phi}, phi in [-pi, pi] (0 for z = 0): the phase
// as one real in [-1, 1].  w = e^{i phi/2} with Re w >= 0 comes from the
// half-angle formulas in whichever form has no cancellation.
template <class T> LGF_HD T quarter_tan(cpx<T> z) {
    const T r2 = norm2(z);
    if (!(r2 > T(0))) return T(0);
    const T ir = rsqrt_nr(r2);
    const T c = z.re * ir, sn = z.im * ir;
    const T h = T(1) / T(2) * (T(1) + fabs(c));
    const T hs = h * rsqrt_nr(h);              // sqrt((1 + |c|)/2) >= 1/sqrt(2)
    const T q = T(0.5) * sn * recip(hs);       // the other half-angle component
    const T wr = c >= T(0) ? hs : fabs(q);
    const T wi = c >= T(0) ? q : copysign(hs, sn);
    return wi * recip(T(1) + wr);
}

// e^{i phi} from t = tan(phi/4)
template <class T> LGF_HD cpx<T> phase_of_quarter_tan(T t) {
    const T t2 = t * t, d = recip(T(1) + t2);
    const T hr = (T(1) - t2) * d, hi = T(2) * t * d;  // e^{i phi/2}
    return mk<T>(fma(hr, hr, -hi * hi), T(2) * hr * hi);
}

// sqrt(x) for x >= 0 (0 for x <= 0)
template <class T> LGF_HD T sqrt_nonneg(T x) { return x > T(0) ? x * rsqrt_nr(x) : T(0); }

template <class T> LGF_HD cpx<T> sel3(int j, cpx<T> a, cpx<T> b, cpx<T> c) {
    return j == 0 ? a : (j == 1 ? b : c);
}

template <class T> LGF_HD void link8_encode(const mat3<T> &m, cpx<T> (&u)[4]) {
    const T n0 = norm2(m.e[0][0]), n1 = norm2(m.e[0][1]), n2 = norm2(m.e[0][2]);
    // c0: column of the smallest row-0 entry; c2: the larger of the other two
    const int c0 = (n0 <= n1 && n0 <= n2) ? 0 : (n1 <= n2 ? 1 : 2);
    const int j = c0 == 0 ? 1 : 0, k = c0 == 2 ? 1 : 2;
    const T nj = c0 == 0 ? n1 : n0, nk = c0 == 2 ? n1 : n2;
    const int c2 = nk > nj ? k : j, c1 = 3 - c0 - c2;
    const bool odd = c2 == (c0 == 2 ? 0 : c0 + 1);  // (c0, c1, c2) not a cyclic shift
    const cpx<T> x10 = sel3(c0, m.e[1][0], m.e[1][1], m.e[1][2]);
    const cpx<T> x20 = sel3(c0, m.e[2][0], m.e[2][1], m.e[2][2]);
    const bool swap = norm2(x10) > norm2(x20);
    const cpx<T> v01 = sel3(c1, m.e[0][0], m.e[0][1], m.e[0][2]);
    u[0] = sel3(c0, m.e[0][0], m.e[0][1], m.e[0][2]);
    u[1] = mk<T>(with_tag(v01.re, c0), with_tag(v01.im, (odd ? 1 : 0) | (swap ? 2 : 0)));
    u[2] = swap ? x20 : x10;
    u[3] = mk<T>(quarter_tan(sel3(c2, m.e[0][0], m.e[0][1], m.e[0][2])),
                 quarter_tan(swap ? x10 : x20));
}

template <class T> LGF_HD mat3<T> link8_decode(const cpx<T> (&u)[4]) {
    const int t0 = tag_of(u[1].re), bits = tag_of(u[1].im);
    const int c0 = t0 > 2 ? 2 : t0;
    const bool odd = (bits & 1) != 0, swap = (bits & 2) != 0;
    const int c2 = odd ? (c0 == 2 ? 0 : c0 + 1) : (c0 == 0 ? 2 : c0 - 1);
    const int c1 = 3 - c0 - c2;
    const cpx<T> a0 = u[0], a1 = mk<T>(untag(u[1].re), untag(u[1].im)), b0 = u[2];
    const T n0 = norm2(a0);
    const cpx<T> a2 = sqrt_nonneg(T(1) - n0 - norm2(a1)) * phase_of_quarter_tan(u[3].re);
    const cpx<T> cc = sqrt_nonneg(T(1) - n0 - norm2(b0)) * phase_of_quarter_tan(u[3].im);
    const T inv = recip(T(1) - n0);
    const T d = odd != swap ? T(-1) : T(1);  // det of the frame V
    // V11 = -(conj(a0) a1 b0 + d conj(a2) conj(cc)) / (1 - |a0|^2)
    // V12 = (d conj(a1) conj(cc) - conj(a0) a2 b0) / (1 - |a0|^2)
    // V21 = d (conj(a2) conj(b0) - conj(a0) conj(V12))
    // V22 = d (conj(a0) conj(V11) - conj(a1) conj(b0))
    const cpx<T> ab = cmul(a1, b0), a2b = cmul(a2, b0);
    const cpx<T> ac = conjg(cmul(a2, cc)), a1c = conjg(cmul(a1, cc));
    const cpx<T> v11 = (-inv) * (cmulc(ab, a0) + d * ac);
    const cpx<T> v12 = inv * (d * a1c - cmulc(a2b, a0));
    const cpx<T> v21 = d * (conjg(cmul(a2, b0)) - conjg(cmul(a0, v12)));
    const cpx<T> v22 = d * (conjg(cmul(a0, v11)) - conjg(cmul(a1, b0)));
    // undo the row swap, then the column permutation (V column k is U column ck)
    const cpx<T> r1[3] = {swap ? cc : b0, swap ? v21 : v11, swap ? v22 : v12};
    const cpx<T> r2[3] = {swap ? b0 : cc, swap ? v11 : v21, swap ? v12 : v22};
    const cpx<T> r0[3] = {a0, a1, a2};
    mat3<T> m;
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const int src = col == c0 ? 0 : (col == c1 ? 1 : 2);
        m.e[0][col] = sel3(src, r0[0], r0[1], r0[2]);
        m.e[1][col] = sel3(src, r1[0], r1[1], r1[2]);
        m.e[2][col] = sel3(src, r2[0], r2[1], r2[2]);
    }
    return m;
}

// ------------------------------------------------------------------------
// Storage layouts
//   links SoA:     L[(mu*LF/2 + k)*S + s], LF/2 complex slots per link for
//                  the link format LF (reals per link):
//                  LF = 12: rows 0,1 (k = 3*row + col); row 2 rebuilt as
//                           conj(row0 x row1) -- the paper's 12-real form
//                  LF = 18: all three rows (no rebuild)
//                  LF = 8:  the minimal form above (4 slots)
//   Fourier field: D[f*S + s], f = 0..3 holding the independent entries of
//                  an anti-hermitian traceless matrix:
//                  f0 = M01, f1 = M02, f2 = M12,
//                  f3 = (Im M00) + i (Im M11)
// ------------------------------------------------------------------------

// rows formed by products when a link is computed for storage in format LF
// (the rest rebuilt): all three for the 18-real form
template <int LF> constexpr int product_rows() { return LF == 18 ? 3 : 2; }

template <class T, int LF> LGF_HD mat3<T> link_from_slots(const cpx<T> (&u)[LF / 2]) {
    if constexpr (LF == 8) {
        return link8_decode<T>(u);
    } else {
        mat3<T> m;
#pragma unroll
        for (int k = 0; k < LF / 2; ++k) m.e[k / 3][k % 3] = u[k];
        if constexpr (LF == 12) rebuild_row2(m);
        return m;
    }
}

template <class T, int LF> LGF_HD void link_to_slots(const mat3<T> &m, cpx<T> (&u)[LF / 2]) {
    if constexpr (LF == 8) {
        link8_encode<T>(m, u);
    } else {
#pragma unroll
        for (int k = 0; k < LF / 2; ++k) u[k] = m.e[k / 3][k % 3];
    }
}

// the link as it reads back after storage in format LF
template <class T, int LF> LGF_HD mat3<T> as_stored(const mat3<T> &m) {
    cpx<T> u[LF / 2];
    link_to_slots<T, LF>(m, u);
    return link_from_slots<T, LF>(u);
}

template <class T, int LF = 12>
LGF_HD mat3<T> load_link(const vec2_t<T> *__restrict__ L, long S, int mu, long s) {
    cpx<T> u[LF / 2];
    const vec2_t<T> *p = L + (long)mu * (LF / 2) * S + s;
#pragma unroll
    for (int k = 0; k < LF / 2; ++k) u[k] = ld<T>(p + (long)k * S);
    return link_from_slots<T, LF>(u);
}

template <class T, int LF = 12>
LGF_HD void store_link(vec2_t<T> *__restrict__ L, long S, int mu, long s, const mat3<T> &m) {
    cpx<T> u[LF / 2];
    link_to_slots<T, LF>(m, u);
    vec2_t<T> *p = L + (long)mu * (LF / 2) * S + s;
#pragma unroll
    for (int k = 0; k < LF / 2; ++k) st_stream<T>(p + (long)k * S, u[k]);
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
