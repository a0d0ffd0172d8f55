// Mixed-radix FFT building blocks for the 4D lattice transforms.
//
// * Extents: every n = 2^a 3^b with 2 <= n <= FFT_MAX_EXTENT (256).
// * dft<N, DIR, TL>: an N-point DFT held entirely in registers, fully
//   unrolled, by recursive decimation in time with radix-4/3/2 butterflies.
//   Twiddles come from the table of the lattice axis being transformed,
//   tw[j] = exp(-2 pi i j / TL) for j < TL (TL = that axis's extent, which N
//   divides), built on the host in long double.  DIR = -1:
//   exp(-2 pi i n k / N) (forward), +1: inverse.
// * lds_axis_fft: transforms every column of a tile held in LDS along one
//   lattice axis.  Extents up to 32 take one register pass per column.  Larger
//   extents N = N1*N2 (N1 <= N2 <= 32, fft_split) take two in-place
//   Stockham-like passes; the forward result is then stored in a permuted
//   order (position p = k1*N2 + k2 holds frequency k1 + N1*k2) that the
//   matching inverse takes back to natural order.  Whatever sits between
//   forward and inverse (the momentum-space scaling) only needs each
//   position's frequency, see fft_freq_of_pos.
#pragma once
#include "su3.hpp"

namespace lgf {

constexpr int FFT_MAX_EXTENT = 256;

// N1 of the two-pass split of an extent n > 32: the largest divisor N1 with
// N1 * N1 <= n and n / N1 <= 32 (the most balanced split into two register
// transforms); 1 when n <= 32 or no such split exists.
__host__ __device__ constexpr int fft_split(int n) {
    int best = 1;
    if (n > 32)
        for (int d = 2; d * d <= n; ++d)
            if (n % d == 0 && n / d <= 32) best = d;
    return best;
}

// complex values one column transform of extent n keeps in registers at a
// time: the whole column up to 32, else the larger factor of its split
__host__ __device__ constexpr int fft_reg_span(int n) {
    return n <= 32 ? n : n / fft_split(n);
}

// Register tier of an extent: the kernels that transform along a runtime
// extent are instantiated per tier, and an instance's register allocation is
// that of the heaviest transform it holds.  Tier 16: one-pass extents up to
// 16 and two-pass extents N1 x N2 with N1 <= 8, N2 <= 12 (36 = 6x6,
// 48 = 6x8, 54 = 6x9, 64 = 8x8, 72 = 8x9, 96 = 8x12), which fit 128 VGPRs
// in every pass kernel; tier 32: the rest.
__host__ __device__ constexpr int fft_tier(int n) {
    return n <= 32 ? (n <= 16 ? 16 : 32)
                   : ((fft_split(n) <= 8 && n / fft_split(n) <= 12) ? 16 : 32);
}

__host__ __device__ constexpr bool fft_supported(int n) {
    if (n < 2 || n > FFT_MAX_EXTENT) return false;
    int m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1 && (n <= 32 || fft_split(n) > 1);
}

// frequency held at position p after a forward transform of extent n
__host__ __device__ constexpr int fft_freq_of_pos(int n, int p) {
    return n <= 32 ? p : (p / (n / fft_split(n))) + fft_split(n) * (p % (n / fft_split(n)));
}

template <int N, int DIR, class T, int TL>
LGF_HD cpx<T> twiddle(const vec2_t<T> *__restrict__ tw, int k) {
    // W_N^k = exp(DIR * 2 pi i k / N) from the axis table of length TL
    static_assert(TL % N == 0, "the transform length must divide the table length");
    vec2_t<T> w = tw[((k % N) + N) % N * (TL / N)];
    return DIR < 0 ? mk<T>(w.x, w.y) : mk<T>(w.x, -w.y);
}

template <int DIR, class T> LGF_HD void bfly2(cpx<T> *a) {
    cpx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
}

template <int DIR, class T> LGF_HD void bfly3(cpx<T> *a) {
    // W3 = exp(DIR 2 pi i / 3) = -1/2 + i DIR sqrt(3)/2
    const T h = T(0.86602540378443864676372317075293618);
    cpx<T> s = a[1] + a[2], d = a[1] - a[2];
    cpx<T> m = a[0] - T(0.5) * s;
    cpx<T> r = mk<T>(-T(DIR) * h * d.im, T(DIR) * h * d.re);  // i DIR h d
    a[0] = a[0] + s;
    a[1] = m + r;
    a[2] = m - r;
}

template <int DIR, class T> LGF_HD void bfly4(cpx<T> *a) {
    cpx<T> s02 = a[0] + a[2], d02 = a[0] - a[2];
    cpx<T> s13 = a[1] + a[3], d13 = a[1] - a[3];
    cpx<T> r = mk<T>(-T(DIR) * d13.im, T(DIR) * d13.re);  // i DIR d13
    a[0] = s02 + s13;
    a[2] = s02 - s13;
    a[1] = d02 + r;
    a[3] = d02 - r;
}

template <int N, int DIR, int TL = N, class T>
LGF_HD void dft(cpx<T> *a, const vec2_t<T> *__restrict__ tw) {
    if constexpr (N == 1) {
        return;
    } else if constexpr (N == 2) {
        bfly2<DIR>(a);
    } else if constexpr (N == 3) {
        bfly3<DIR>(a);
    } else if constexpr (N == 4) {
        bfly4<DIR>(a);
    } else {
        constexpr int P = (N % 4 == 0) ? 4 : ((N % 3 == 0) ? 3 : 2);
        constexpr int Q = N / P;
        cpx<T> b[P][Q];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int m = 0; m < Q; ++m) b[p][m] = a[m * P + p];
#pragma unroll
        for (int p = 0; p < P; ++p) dft<Q, DIR, TL>(b[p], tw);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            cpx<T> t[P];
            t[0] = b[0][k];
#pragma unroll
            for (int p = 1; p < P; ++p)
                t[p] = (k == 0) ? b[p][k] : cmul(b[p][k], twiddle<N, DIR, T, TL>(tw, p * k));
            if constexpr (P == 4) bfly4<DIR>(t);
            else if constexpr (P == 3) bfly3<DIR>(t);
            else bfly2<DIR>(t);
#pragma unroll
            for (int s = 0; s < P; ++s) a[k + Q * s] = t[s];
        }
    }
}

// Column c of the tile: elements lds[base(c) + j*stride], j < N.
// Must be called by every thread of the block (two-pass extents synchronise).
template <int N, int DIR, class T, class Base>
LGF_HD void lds_axis_fft_n(vec2_t<T> *lds, int ncols, int stride, Base base,
                           const vec2_t<T> *__restrict__ tw) {
    const int nthr = blockDim.x;
    if constexpr (N <= 32) {
        for (int c = threadIdx.x; c < ncols; c += nthr) {
            const int b0 = base(c);
            cpx<T> a[N];
#pragma unroll
            for (int j = 0; j < N; ++j) a[j] = ld<T>(lds + b0 + j * stride);
            dft<N, DIR, N>(a, tw);
#pragma unroll
            for (int j = 0; j < N; ++j) st<T>(lds + b0 + j * stride, a[j]);
        }
    } else {
        constexpr int N1 = fft_split(N), N2 = N / N1;
        static_assert(N1 * N2 == N && N1 > 1, "unsupported extent");
        if constexpr (DIR < 0) {
            // pass 1: for each n2, DFT_N1 over n1 (stride N2), times W_N^(n2 k1)
            for (int w = threadIdx.x; w < ncols * N2; w += nthr) {
                const int c = w / N2, n2 = w - c * N2;
                const int b0 = base(c) + n2 * stride;
                cpx<T> a[N1];
#pragma unroll
                for (int j = 0; j < N1; ++j) a[j] = ld<T>(lds + b0 + j * N2 * stride);
                dft<N1, DIR, N>(a, tw);
#pragma unroll
                for (int k1 = 1; k1 < N1; ++k1) a[k1] = cmul(a[k1], twiddle<N, DIR, T, N>(tw, n2 * k1));
#pragma unroll
                for (int j = 0; j < N1; ++j) st<T>(lds + b0 + j * N2 * stride, a[j]);
            }
            __syncthreads();
            // pass 2: for each k1, DFT_N2 over n2 (contiguous block of N2)
            for (int w = threadIdx.x; w < ncols * N1; w += nthr) {
                const int c = w / N1, k1 = w - c * N1;
                const int b0 = base(c) + k1 * N2 * stride;
                cpx<T> a[N2];
#pragma unroll
                for (int j = 0; j < N2; ++j) a[j] = ld<T>(lds + b0 + j * stride);
                dft<N2, DIR, N>(a, tw);
#pragma unroll
                for (int j = 0; j < N2; ++j) st<T>(lds + b0 + j * stride, a[j]);
            }
        } else {
            // undo pass 2: for each k1, inverse DFT_N2 over the block, times W_N^(-n2 k1)
            for (int w = threadIdx.x; w < ncols * N1; w += nthr) {
                const int c = w / N1, k1 = w - c * N1;
                const int b0 = base(c) + k1 * N2 * stride;
                cpx<T> a[N2];
#pragma unroll
                for (int j = 0; j < N2; ++j) a[j] = ld<T>(lds + b0 + j * stride);
                dft<N2, DIR, N>(a, tw);
#pragma unroll
                for (int n2 = 1; n2 < N2; ++n2) a[n2] = cmul(a[n2], twiddle<N, DIR, T, N>(tw, n2 * k1));
#pragma unroll
                for (int j = 0; j < N2; ++j) st<T>(lds + b0 + j * stride, a[j]);
            }
            __syncthreads();
            // undo pass 1: for each n2, inverse DFT_N1 over k1 (stride N2)
            for (int w = threadIdx.x; w < ncols * N2; w += nthr) {
                const int c = w / N2, n2 = w - c * N2;
                const int b0 = base(c) + n2 * stride;
                cpx<T> a[N1];
#pragma unroll
                for (int j = 0; j < N1; ++j) a[j] = ld<T>(lds + b0 + j * N2 * stride);
                dft<N1, DIR, N>(a, tw);
#pragma unroll
                for (int j = 0; j < N1; ++j) st<T>(lds + b0 + j * N2 * stride, a[j]);
            }
        }
    }
}

// Column transform forward, times scale(prep(c), position), inverse, in place.
// Extents up to 32 take one register pass per column.  Two-pass extents take
// the forward pass 1, then per (column, k1) the forward N2-point DFT, the
// scaling and the inverse N2-point DFT with its twiddles in registers, then
// the inverse pass 1: two LDS round trips and two barriers fewer than a
// forward transform, a scaling pass and an inverse transform, with the same
// arithmetic in the same order.  Must be called by every thread of the block.
template <int N, class T, class Base, class Prep, class Scale>
LGF_HD void lds_axis_fsi_n(vec2_t<T> *lds, int ncols, int stride, Base base, Prep prep,
                           Scale scale, const vec2_t<T> *__restrict__ tw) {
    const int nthr = blockDim.x;
    if constexpr (N <= 32) {
        for (int c = threadIdx.x; c < ncols; c += nthr) {
            const int b0 = base(c);
            const auto info = prep(c);
            cpx<T> a[N];
#pragma unroll
            for (int j = 0; j < N; ++j) a[j] = ld<T>(lds + b0 + j * stride);
            dft<N, -1, N>(a, tw);
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const T f = scale(info, k);
                a[k].re *= f;
                a[k].im *= f;
            }
            dft<N, +1, N>(a, tw);
#pragma unroll
            for (int j = 0; j < N; ++j) st<T>(lds + b0 + j * stride, a[j]);
        }
    } else {
        constexpr int N1 = fft_split(N), N2 = N / N1;
        static_assert(N1 * N2 == N && N1 > 1, "unsupported extent");
        // forward pass 1: for each n2, DFT_N1 over n1 (stride N2), times W_N^(n2 k1)
        for (int w = threadIdx.x; w < ncols * N2; w += nthr) {
            const int c = w / N2, n2 = w - c * N2;
            const int b0 = base(c) + n2 * stride;
            cpx<T> a[N1];
#pragma unroll
            for (int j = 0; j < N1; ++j) a[j] = ld<T>(lds + b0 + j * N2 * stride);
            dft<N1, -1, N>(a, tw);
#pragma unroll
            for (int k1 = 1; k1 < N1; ++k1) a[k1] = cmul(a[k1], twiddle<N, -1, T, N>(tw, n2 * k1));
#pragma unroll
            for (int j = 0; j < N1; ++j) st<T>(lds + b0 + j * N2 * stride, a[j]);
        }
        __syncthreads();
        // per k1: forward DFT_N2 (position k1 N2 + k2), scaling, inverse DFT_N2,
        // times W_N^(-n2 k1)
        for (int w = threadIdx.x; w < ncols * N1; w += nthr) {
            const int c = w / N1, k1 = w - c * N1;
            const int b0 = base(c) + k1 * N2 * stride;
            const auto info = prep(c);
            cpx<T> a[N2];
#pragma unroll
            for (int j = 0; j < N2; ++j) a[j] = ld<T>(lds + b0 + j * stride);
            dft<N2, -1, N>(a, tw);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) {
                const T f = scale(info, k1 * N2 + k2);
                a[k2].re *= f;
                a[k2].im *= f;
            }
            dft<N2, +1, N>(a, tw);
#pragma unroll
            for (int n2 = 1; n2 < N2; ++n2) a[n2] = cmul(a[n2], twiddle<N, +1, T, N>(tw, n2 * k1));
#pragma unroll
            for (int j = 0; j < N2; ++j) st<T>(lds + b0 + j * stride, a[j]);
        }
        __syncthreads();
        // inverse pass 1: for each n2, inverse DFT_N1 over k1 (stride N2)
        for (int w = threadIdx.x; w < ncols * N2; w += nthr) {
            const int c = w / N2, n2 = w - c * N2;
            const int b0 = base(c) + n2 * stride;
            cpx<T> a[N1];
#pragma unroll
            for (int j = 0; j < N1; ++j) a[j] = ld<T>(lds + b0 + j * N2 * stride);
            dft<N1, +1, N>(a, tw);
#pragma unroll
            for (int j = 0; j < N1; ++j) st<T>(lds + b0 + j * N2 * stride, a[j]);
        }
    }
}

// Every supported extent (fft_supported), as MACRO(n) for each.
#define LGF_FFT_SMALL_EXTENTS(MACRO)                                                     \
    MACRO(2) MACRO(3) MACRO(4) MACRO(6) MACRO(8) MACRO(9) MACRO(12) MACRO(16) MACRO(18)  \
    MACRO(24) MACRO(27) MACRO(32)
#define LGF_FFT_EXTENTS(MACRO)                                                           \
    LGF_FFT_SMALL_EXTENTS(MACRO)                                                         \
    MACRO(36) MACRO(48) MACRO(54) MACRO(64) MACRO(72) MACRO(81) MACRO(96) MACRO(108)     \
    MACRO(128) MACRO(144) MACRO(162) MACRO(192) MACRO(216) MACRO(243) MACRO(256)

template <class T, int RMAX, class Base, class Prep, class Scale>
LGF_HD void lds_axis_fsi(int n, vec2_t<T> *lds, int ncols, int stride, Base base, Prep prep,
                         Scale scale, const vec2_t<T> *__restrict__ tw) {
    switch (n) {
#define LGF_CASE(NN)                                                                   \
    case NN:                                                                           \
        if constexpr (fft_tier(NN) <= RMAX)                                            \
            lds_axis_fsi_n<NN, T>(lds, ncols, stride, base, prep, scale, tw);          \
        break;
        LGF_FFT_EXTENTS(LGF_CASE)
#undef LGF_CASE
    default: break;
    }
}

// Runtime-extent dispatch over the extents of register tier at most RMAX
// (fft_tier): a kernel's register allocation is that of its largest case, so
// a kernel instantiated for tier 16 runs at a higher occupancy.
template <int DIR, class T, int RMAX, class Base>
LGF_HD void lds_axis_fft(int n, vec2_t<T> *lds, int ncols, int stride, Base base,
                         const vec2_t<T> *__restrict__ tw) {
    switch (n) {
#define LGF_CASE(NN)                                                                   \
    case NN:                                                                           \
        if constexpr (fft_tier(NN) <= RMAX)                                            \
            lds_axis_fft_n<NN, DIR, T>(lds, ncols, stride, base, tw);                  \
        break;
        LGF_FFT_EXTENTS(LGF_CASE)
#undef LGF_CASE
    default: break;
    }
}

}  // namespace lgf
