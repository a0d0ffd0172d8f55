// FFT pass kernels and their launchers, templated on the real type.  The
// translation units fft_f64.hip and fft_f32.hip instantiate them.
//
//   k_fft_xy_rc / k_fft_zt_rc  one axis held in registers, the other
//                              exchanged through LDS (extents <= 32)
//   k_fft_xy                   a whole (x,y) plane in LDS (larger extents)
//   k_fft_axis                 one axis of the (z,t) plane per pass, W sites
//                              x the axis x B slices in LDS (larger extents)
#pragma once
#include <type_traits>

#include "common.hpp"

namespace lgf {

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

// 1/x from the hardware estimate refined by Newton steps (to about 1 ulp).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Momentum-space factor p2max/(V p2) of one (z,t) column: `base` is the
// column's p2 without the z term (negative for a padding column).
template <class T>
__device__ __forceinline__ T fa_factor(T base, T pz, T p2max_over_V) {
    const T p2 = base + pz;
    return (base < T(0) || p2 == T(0)) ? T(0) : p2max_over_V * recip(p2);
}

// ---------------------------------------------------------------------------
// (x, y) plane transform: one plane of one field per block, LDS [y][x+1]
// ---------------------------------------------------------------------------

constexpr int XY_BLOCK = 256;

// RMAX: largest register span (fft_reg_span) of the extents this instance handles
template <class T, int DIR, int RMAX>
__global__ void __launch_bounds__(XY_BLOCK)
    k_fft_xy(geom g, vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ tw,
             const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    const int Lx = g.Lx, Ly = g.Ly, P = Lx + 1;
    const long Lxy = (long)Lx * Ly;
    vec2_t<T> *plane = D + (long)blockIdx.y * g.S + (long)blockIdx.x * Lxy;
    for (int i = threadIdx.x; i < Lxy; i += XY_BLOCK) {
        const int y = i / Lx, x = i - y * Lx;
        lds[y * P + x] = plane[i];
    }
    __syncthreads();
    auto rows = [P](int c) { return c * P; };
    auto cols = [](int c) { return c; };
    if (DIR < 0) {
        lds_axis_fft<DIR, T, RMAX>(Lx, lds, Ly, 1, rows, tw);
        __syncthreads();
        lds_axis_fft<DIR, T, RMAX>(Ly, lds, Lx, P, cols, tw);
    } else {
        lds_axis_fft<DIR, T, RMAX>(Ly, lds, Lx, P, cols, tw);
        __syncthreads();
        lds_axis_fft<DIR, T, RMAX>(Lx, lds, Ly, 1, rows, tw);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Lxy; i += XY_BLOCK) {
        const int y = i / Lx, x = i - y * Lx;
        plane[i] = lds[y * P + x];
    }
}

// Inverse (x, y) pass of the FP32 sweeps of an SU(3) mixed solve on planes
// wider than 32, fused with G(x) <- g(x) G(x): one plane of all 4 fields per
// block (4 LDS regions [y][x+1]); after the transform each site's 4 entries
// of L Delta are read from the regions, g is formed and G goes from Gold into
// Gnew.  L Delta itself is not stored.
template <class T, int RMAX, bool EXACT>
__global__ void __launch_bounds__(XY_BLOCK)
    k_fft_xy_acc(geom g, const vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ tw,
                 const vec2_t<T> *__restrict__ Gold, vec2_t<T> *__restrict__ Gnew, double c,
                 const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    const int Lx = g.Lx, Ly = g.Ly, P = Lx + 1, REG = Ly * P;
    const int Lxy = Lx * Ly;
    const long s0 = (long)blockIdx.x * Lxy;
    for (int f = 0; f < 4; ++f)
        for (int i = threadIdx.x; i < Lxy; i += XY_BLOCK) {
            const int y = i / Lx, x = i - y * Lx;
            lds[f * REG + y * P + x] = D[(long)f * g.S + s0 + i];
        }
    __syncthreads();
    auto cols = [Lx, REG](int cc) { return (cc / Lx) * REG + (cc % Lx); };      // cc = x + Lx f
    auto rows = [Ly, REG, P](int cc) { return (cc / Ly) * REG + (cc % Ly) * P; };  // cc = y + Ly f
    lds_axis_fft<+1, T, RMAX>(Ly, lds, 4 * Lx, P, cols, tw);
    __syncthreads();
    lds_axis_fft<+1, T, RMAX>(Lx, lds, 4 * Ly, 1, rows, tw);
    __syncthreads();
    for (int i = threadIdx.x; i < Lxy; i += XY_BLOCK) {
        const int y = i / Lx, x = i - y * Lx;
        const vec2_t<T> *q = lds + y * P + x;
        accumulate_G<EXACT>(ld<T>(q), ld<T>(q + REG), ld<T>(q + 2 * REG), ld<T>(q + 3 * REG), c,
                            Gold, Gnew, g.S, s0 + i);
    }
}

// ---------------------------------------------------------------------------
// One-axis passes for (z, t) planes too large for a register column (an
// extent above 32): the (z,t) transform becomes three passes over the field,
// z forward, then t forward / scaling / t inverse, then z inverse.  A block
// holds W consecutive xy-sites (rows of up to 1 KB) x the whole axis x B
// slices of the other axis, so every load and store is a coalesced row;
// the transform of each column runs in LDS (lds_axis_fft, one or two passes).
// LDS element (w, j, b) at b*N*PW + j*PW + w, PW = W + 1.
// AX = 2: the z axis (slices along t); AX = 3: the t axis (slices along z).
// MODE -1 forward, +1 inverse, 0 (t axis only) forward, times p2max/(V p2),
// inverse.
// ---------------------------------------------------------------------------

constexpr int AXIS_BLOCK = 256;
constexpr int ZT_PAD = 4;

// Register budgets: 128 VGPRs for spans up to 16 (four waves per SIMD, the
// occupancy the 32 KB tiles allow; the fused scaled round trip would take
// 129), 256 for the wider spans (without the hint it spills to AGPRs).
template <class T, int AX, int MODE, int RMAX>
__global__ void __launch_bounds__(AXIS_BLOCK) __attribute__((amdgpu_waves_per_eu(RMAX <= 16 ? 4 : 2)))
    k_fft_axis(geom g, vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ tw,
               const T *__restrict__ ptab, T p2max_over_V, int W, int B,
               const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    const int Lz = g.Lz, N = AX == 2 ? g.Lz : g.Lt;
    const long Lxy = (long)g.Lx * g.Ly;
    const long s0 = (long)xcd_block(blockIdx.x, gridDim.x) * W;
    const int Wt = (int)min((long)W, Lxy - s0);
    const int o0 = blockIdx.y * B;  // first slice of the other axis
    const int PW = W + 1, PB = N * PW;
    vec2_t<T> *F = D + (long)blockIdx.z * g.S + s0;
    // (z, t) plane index of element (j, b)
    auto zt = [=](int j, int b) { return AX == 2 ? (o0 + b) * Lz + j : j * Lz + (o0 + b); };
    const int nel = W * N * B;
    for (int i = threadIdx.x; i < nel; i += AXIS_BLOCK) {
        const int w = i % W, r = i / W, j = r % N, b = r / N;
        vec2_t<T> v;
        v.x = 0;
        v.y = 0;
        if (w < Wt) v = F[(long)zt(j, b) * Lxy + w];
        lds[b * PB + j * PW + w] = v;
    }
    __syncthreads();
    auto col = [W, PW, PB](int c) { return (c / W) * PB + (c % W); };  // c = w + W*b
    if (MODE == 0) {
        const T *px = ptab, *py = ptab + g.Lx, *pz = ptab + g.Lx + g.Ly,
                *pt = ptab + g.Lx + g.Ly + g.Lz;
        // per column c = w + W*b: its p2 without the t term, or -1 for a
        // padding column of a ragged tile (factor 0)
        auto prep = [=](int c) -> T {
            const int w = c % W, b = c / W;
            const long sxy = s0 + w;
            if (sxy >= Lxy) return T(-1);
            const int y = (int)(sxy / g.Lx), x = (int)(sxy - (long)y * g.Lx);
            return (px[x] + py[y]) + pz[o0 + b];
        };
        auto scale = [=](T base, int j) -> T { return fa_factor<T>(base, pt[j], p2max_over_V); };
        lds_axis_fsi<T, RMAX>(N, lds, W * B, PW, col, prep, scale, tw);
    } else {
        lds_axis_fft<MODE, T, RMAX>(N, lds, W * B, PW, col, tw);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nel; i += AXIS_BLOCK) {
        const int w = i % W, r = i / W, j = r % N, b = r / N;
        if (w < Wt) F[(long)zt(j, b) * Lxy + w] = lds[b * PB + j * PW + w];
    }
}

// ---------------------------------------------------------------------------
// Register-column transforms (register-axis extent up to 32).
//
// Each thread keeps the whole column of one strided lattice axis (t for the
// (z,t) pass, y for the (x,y) pass) in registers, loaded straight from HBM so
// that consecutive lanes read consecutive sites.  The other axis is
// transformed through LDS: every thread writes its whole column, the columns
// of the exchanged axis are transformed by all threads at once, and the values
// are read back (the register copy is dead meanwhile, which keeps the register
// peak down).  LDS element (w, b, j) is at j*PJ + b*SB + w*SW; the tile width
// is chosen on the host so that the tile fits the LDS budget.
// ---------------------------------------------------------------------------


template <int NA, class T, class ColFn>
__device__ __forceinline__ void exchange_axis(cpx<T> (&a)[NA], int w, int b, int SB, int SW,
                                              int PJ, vec2_t<T> *lds, ColFn col) {
    vec2_t<T> *mine = lds + b * SB + w * SW;
#pragma unroll
    for (int j = 0; j < NA; ++j) st<T>(mine + j * PJ, a[j]);
    __syncthreads();
    col(0, NA);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NA; ++j) a[j] = ld<T>(mine + j * PJ);
}

// Column transform forward, times scale(info, position), inverse, in one
// register pass (extent up to 32); info = prep(c) is computed once per column.
template <int N, class T, class Base, class Prep, class Scale>
__device__ __forceinline__ void col_fwd_scale_inv_n(vec2_t<T> *lds, int ncols, int stride, Base base,
                                                    Prep prep, Scale scale,
                                                    const vec2_t<T> *__restrict__ tw) {
    for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
        const int b0 = base(c);
        const auto info = prep(c);
        cpx<T> v[N];
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = ld<T>(lds + b0 + k * stride);
        dft<N, -1>(v, tw);
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = scale(info, k) * v[k];
        dft<N, +1>(v, tw);
#pragma unroll
        for (int k = 0; k < N; ++k) st<T>(lds + b0 + k * stride, v[k]);
    }
}

template <class T, class Base, class Prep, class Scale>
__device__ __forceinline__ void col_fwd_scale_inv(int n, vec2_t<T> *lds, int ncols, int stride,
                                                  Base base, Prep prep, Scale scale,
                                                  const vec2_t<T> *__restrict__ tw) {
    switch (n) {
#define LGF_SCASE(NN) \
    case NN: col_fwd_scale_inv_n<NN, T>(lds, ncols, stride, base, prep, scale, tw); break;
        LGF_SCASE(2) LGF_SCASE(3) LGF_SCASE(4) LGF_SCASE(6) LGF_SCASE(8) LGF_SCASE(12)
        LGF_SCASE(16) LGF_SCASE(24) LGF_SCASE(32)
#undef LGF_SCASE
    default: break;
    }
}

// One-pass column transform of an extent up to 32.
template <int DIR, class T, class Base>
__device__ __forceinline__ void col_fft_small(int n, vec2_t<T> *lds, int ncols, int stride,
                                              Base base, const vec2_t<T> *__restrict__ tw) {
    switch (n) {
#define LGF_CCASE(NN) \
    case NN: lds_axis_fft_n<NN, DIR, T>(lds, ncols, stride, base, tw); break;
        LGF_CCASE(2) LGF_CCASE(3) LGF_CCASE(4) LGF_CCASE(6) LGF_CCASE(8) LGF_CCASE(12)
        LGF_CCASE(16) LGF_CCASE(24) LGF_CCASE(32)
#undef LGF_CCASE
    default: break;
    }
}

template <class T> constexpr int rc_max_threads() { return sizeof(T) == 8 ? 256 : 512; }

// (x, y) pass: F fields of one plane per block, thread (f, x) holds a y-column.
template <class T, int NY, int DIR>
__global__ void __launch_bounds__(rc_max_threads<T>())
    k_fft_xy_rc(geom g, vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ tw, int F,
                const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    const int Lx = g.Lx;
    const long Lxy = (long)Lx * NY;
    const int x = threadIdx.x % Lx, fl = threadIdx.x / Lx;
    const int f = blockIdx.y * F + fl;
    const int SW = Lx + 1, PJ = F * SW;
    vec2_t<T> *p = D + (long)f * g.S + (long)blockIdx.x * Lxy + x;
    cpx<T> a[NY];
#pragma unroll
    for (int y = 0; y < NY; ++y) a[y] = ld<T>(p + (long)y * Lx);
    auto base = [F, SW, PJ](int c) { return (c / F) * PJ + (c % F) * SW; };  // c = fl + F*j
    auto col = [&](int, int C) { col_fft_small<DIR, T>(Lx, lds, F * C, 1, base, tw); };
    if (DIR < 0) {
        dft<NY, -1>(a, tw);
        exchange_axis<NY, T>(a, fl, x, 1, SW, PJ, lds, col);
    } else {
        exchange_axis<NY, T>(a, fl, x, 1, SW, PJ, lds, col);
        dft<NY, +1>(a, tw);
    }
#pragma unroll
    for (int y = 0; y < NY; ++y) st<T>(p + (long)y * Lx, a[y]);
}

// Inverse (x, y) pass of the FP32 sweeps of an SU(3) mixed solve, fused with
// the accumulation G(x) <- g(x) G(x): the block holds all 4 fields of its
// plane, so after the inverse transform each site's 4 entries of L Delta are
// gathered through LDS, g is formed (first-order or exact step, coefficient
// c) and G is updated from Gold into Gnew.  L Delta itself is not stored (the
// update reads only G).
template <class T, int NY, bool EXACT>
__global__ void __launch_bounds__(rc_max_threads<T>())
    k_fft_xy_rc_acc(geom g, const vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ tw,
                    const vec2_t<T> *__restrict__ Gold, vec2_t<T> *__restrict__ Gnew, double c,
                    const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    constexpr int F = 4;
    const int Lx = g.Lx;
    const long Lxy = (long)Lx * NY;
    const int x = threadIdx.x % Lx, fl = threadIdx.x / Lx;
    const int SW = Lx + 1, PJ = F * SW;
    const vec2_t<T> *p = D + (long)fl * g.S + (long)blockIdx.x * Lxy + x;
    cpx<T> a[NY];
#pragma unroll
    for (int y = 0; y < NY; ++y) a[y] = ld<T>(p + (long)y * Lx);
    auto base = [SW, PJ](int cc) { return (cc / F) * PJ + (cc % F) * SW; };  // cc = fl + F*j
    auto col = [&](int, int C) { col_fft_small<+1, T>(Lx, lds, F * C, 1, base, tw); };
    exchange_axis<NY, T>(a, fl, x, 1, SW, PJ, lds, col);
    dft<NY, +1>(a, tw);
    __syncthreads();  // every thread has read its column back
#pragma unroll
    for (int y = 0; y < NY; ++y) st<T>(lds + y * PJ + fl * SW + x, a[y]);
    __syncthreads();
    const long s0 = (long)blockIdx.x * Lxy;
    for (int i = threadIdx.x; i < (int)Lxy; i += blockDim.x) {
        const int y = i / Lx, xx = i - y * Lx;
        const vec2_t<T> *q = lds + y * PJ + xx;
        accumulate_G<EXACT>(ld<T>(q), ld<T>(q + SW), ld<T>(q + 2 * SW), ld<T>(q + 3 * SW), c, Gold,
                            Gnew, g.S, s0 + i);
    }
}

// (z, t) pass: W consecutive xy-sites of one field per block, thread (w, z)
// holds a t-column.  MODE 0: forward, scale by p2max/(V p2), inverse.
template <class T, int NT, int MODE>
__global__ void __launch_bounds__(rc_max_threads<T>())
    k_fft_zt_rc(geom g, vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ tw,
                const T *__restrict__ ptab, T p2max_over_V, int W,
                const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    const int Lz = g.Lz;
    const long Lxy = (long)g.Lx * g.Ly;
    const int w = threadIdx.x % W, z = threadIdx.x / W;
    const long s0 = (long)xcd_block(blockIdx.x, gridDim.x) * W;
    const bool live = s0 + w < Lxy;
    vec2_t<T> *p = D + (long)blockIdx.y * g.S + (long)z * Lxy + s0 + w;
    const long tstride = (long)Lz * Lxy;
    cpx<T> a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = live ? ld<T>(p + t * tstride) : mk<T>(0, 0);
    const int PJ = Lz * W + ZT_PAD;
    auto base = [W, PJ](int c) { return (c / W) * PJ + (c % W); };  // c = w + W*j
    if (MODE <= 0) dft<NT, -1>(a, tw);
    if (MODE == 0) {
        const T *px = ptab, *py = ptab + g.Lx, *pz = ptab + g.Lx + g.Ly,
                *pt = ptab + g.Lx + g.Ly + g.Lz;
        const int Lx = g.Lx, s0i = (int)s0, Lxyi = (int)Lxy;
        auto col = [&](int c0, int C) {
            // column c = w + W*j along z at t position c0 + j
            auto prep = [=](int c) -> T {
                const int sxy = s0i + (c % W);
                if (sxy >= Lxyi) return T(-1);  // padding column of a ragged tile
                const int y = sxy / Lx, x = sxy - y * Lx;
                return (px[x] + py[y]) + pt[c0 + c / W];
            };
            auto scale = [=](T base, int k) -> T { return fa_factor<T>(base, pz[k], p2max_over_V); };
            col_fwd_scale_inv<T>(Lz, lds, W * C, W, base, prep, scale, tw);
        };
        exchange_axis<NT, T>(a, w, z, W, 1, PJ, lds, col);
    } else {
        auto col = [&](int, int C) { col_fft_small<MODE, T>(Lz, lds, W * C, W, base, tw); };
        exchange_axis<NT, T>(a, w, z, W, 1, PJ, lds, col);
    }
    if (MODE >= 0) dft<NT, +1>(a, tw);
    if (live) {
#pragma unroll
        for (int t = 0; t < NT; ++t) st<T>(p + t * tstride, a[t]);
    }
}

#define LGF_NA_CASES(MACRO)                                                        \
    MACRO(2) MACRO(3) MACRO(4) MACRO(6) MACRO(8) MACRO(12) MACRO(16) MACRO(24) MACRO(32)

template <class T> inline int xy_fields_per_block(const geom &g) {
    int F = g.nf;
    while (F > 1 && F * g.Lx > rc_max_threads<T>()) F >>= 1;
    return F;
}

template <class T> inline bool xy_use_rc(const geom &g) { return g.Ly <= 32 && g.Lx <= 32; }

template <class T> size_t fft_xy_lds_bytes(const geom &g) {
    if (xy_use_rc<T>(g))
        return (size_t)g.Ly * xy_fields_per_block<T>(g) * (g.Lx + 1) * sizeof(vec2_t<T>);
    return (size_t)g.Ly * (g.Lx + 1) * sizeof(vec2_t<T>);
}

template <class T>
hipError_t launch_fft_xy(const geom &g, void *D, int dir, const void *tw, const dev_status *status,
                         hipStream_t st) {
    auto Dp = static_cast<vec2_t<T> *>(D);
    auto twp = static_cast<const vec2_t<T> *>(tw);
    const size_t lds = fft_xy_lds_bytes<T>(g);
    if (xy_use_rc<T>(g)) {
        const int F = xy_fields_per_block<T>(g);
        dim3 grid((unsigned)(g.Lz * g.Lt), (unsigned)(g.nf / F));
        const unsigned nt = (unsigned)(F * g.Lx);
#define LGF_XY(NN)                                                                            \
    case NN:                                                                                  \
        if (dir < 0) k_fft_xy_rc<T, NN, -1><<<grid, nt, lds, st>>>(g, Dp, twp, F, status);   \
        else k_fft_xy_rc<T, NN, 1><<<grid, nt, lds, st>>>(g, Dp, twp, F, status);            \
        break;
        switch (g.Ly) {
            LGF_NA_CASES(LGF_XY)
        default: return hipErrorInvalidValue;
        }
#undef LGF_XY
        return hipGetLastError();
    }
    dim3 grid((unsigned)(g.Lz * g.Lt), (unsigned)g.nf);
    if (fft_reg_span(g.Lx) <= 16 && fft_reg_span(g.Ly) <= 16) {
        if (dir < 0) k_fft_xy<T, -1, 16><<<grid, XY_BLOCK, lds, st>>>(g, Dp, twp, status);
        else k_fft_xy<T, +1, 16><<<grid, XY_BLOCK, lds, st>>>(g, Dp, twp, status);
    } else {
        if (dir < 0) k_fft_xy<T, -1, 32><<<grid, XY_BLOCK, lds, st>>>(g, Dp, twp, status);
        else k_fft_xy<T, +1, 32><<<grid, XY_BLOCK, lds, st>>>(g, Dp, twp, status);
    }
    return hipGetLastError();
}

// The fused inverse (x,y) pass with G accumulation: register-column planes
// holding all 4 fields in one block.
constexpr size_t XY_ACC_LDS_MAX = 150 * 1024;
template <class T> inline size_t xy_acc_lds_bytes(const geom &g) {
    return (size_t)4 * g.Ly * (g.Lx + 1) * sizeof(vec2_t<T>);
}
template <class T> inline bool xy_acc_fusable(const geom &g) {
    if (g.nc != 3 || g.nf != 4) return false;
    if (xy_use_rc<T>(g)) return xy_fields_per_block<T>(g) == 4;
    return xy_acc_lds_bytes<T>(g) <= XY_ACC_LDS_MAX;
}

template <class T>
hipError_t launch_fft_xy_inv_acc(const geom &g, void *D, const void *tw, const void *Gold,
                                 void *Gnew, double c, bool exact, const dev_status *status,
                                 hipStream_t st) {
    if (!xy_acc_fusable<T>(g)) return hipErrorInvalidValue;
    auto Dp = static_cast<const vec2_t<T> *>(D);
    auto twp = static_cast<const vec2_t<T> *>(tw);
    auto Go = static_cast<const vec2_t<T> *>(Gold);
    auto Gn = static_cast<vec2_t<T> *>(Gnew);
    if (!xy_use_rc<T>(g)) {
        const size_t b = xy_acc_lds_bytes<T>(g);
        const dim3 grid((unsigned)(g.Lz * g.Lt));
        const bool sm = fft_reg_span(g.Lx) <= 16 && fft_reg_span(g.Ly) <= 16;
#define LGF_XG(R, E) k_fft_xy_acc<T, R, E><<<grid, XY_BLOCK, b, st>>>(g, Dp, twp, Go, Gn, c, status)
        if (sm) {
            if (exact) LGF_XG(16, true);
            else LGF_XG(16, false);
        } else {
            if (exact) LGF_XG(32, true);
            else LGF_XG(32, false);
        }
#undef LGF_XG
        return hipGetLastError();
    }
    const size_t lds = fft_xy_lds_bytes<T>(g);
    const dim3 grid((unsigned)(g.Lz * g.Lt));
    const unsigned nt = (unsigned)(4 * g.Lx);
#define LGF_XA(NN)                                                                            \
    case NN:                                                                                  \
        if (exact)                                                                            \
            k_fft_xy_rc_acc<T, NN, true><<<grid, nt, lds, st>>>(g, Dp, twp, Go, Gn, c, status);  \
        else                                                                                  \
            k_fft_xy_rc_acc<T, NN, false><<<grid, nt, lds, st>>>(g, Dp, twp, Go, Gn, c, status); \
        break;
    switch (g.Ly) {
        LGF_NA_CASES(LGF_XA)
    default: return hipErrorInvalidValue;
    }
#undef LGF_XA
    return hipGetLastError();
}

// (z,t) plan: register-column kernel when Lt <= 32 (tile of W sites with
// 128-byte rows), else the LDS-tile kernel with the widest W that fits.
template <class T> zt_plan plan_zt(const geom &g, size_t lds_budget) {
    zt_plan p{};
    const long Lxy = (long)g.Lx * g.Ly;
    if (g.Lt <= 32 && g.Lz <= 32) {
        auto rc_bytes = [&](int w) {
            return (size_t)g.Lt * ((size_t)g.Lz * w + ZT_PAD) * sizeof(vec2_t<T>);
        };
        int W = 128 / (int)sizeof(vec2_t<T>);
        while (W > 1 && (W * g.Lz > rc_max_threads<T>() || W > Lxy || rc_bytes(W) > lds_budget))
            W >>= 1;
        if (W * g.Lz <= rc_max_threads<T>() && rc_bytes(W) <= 160 * 1024) {
            p.rc = true;
            p.W = W;
            p.lds = rc_bytes(W);
            return p;
        }
    }
    // one-axis passes: rows of up to 1 KB (W consecutive sites), then as many
    // slices of the other axis as keep a tile within AXIS_TILE_BYTES, dividing
    // its extent.  32 KB tiles let four blocks share a compute unit (the
    // register limit of these kernels); 64 KB tiles, with wider rows but three
    // blocks, took 15-25% longer at 48^3 x 96.
    constexpr size_t AXIS_TILE_BYTES = 32 * 1024;
    auto tile = [&](int n, int w, int b) { return (size_t)b * n * (w + 1) * sizeof(vec2_t<T>); };
    auto width = [&](int n) {
        int w = 1024 / (int)sizeof(vec2_t<T>);
        while (w > 1 && (w > Lxy || tile(n, w, 1) > AXIS_TILE_BYTES)) w >>= 1;
        return w;
    };
    auto slices = [&](int n, int w, int other) {
        int b = 8;
        while (b > 1 && (other % b != 0 || tile(n, w, b) > AXIS_TILE_BYTES)) b >>= 1;
        return b;
    };
    p.rc = false;
    p.Wz = width(g.Lz);
    p.Wt = width(g.Lt);
    p.W = p.Wz;
    p.Bz = slices(g.Lz, p.Wz, g.Lt);
    p.Bt = slices(g.Lt, p.Wt, g.Lz);
    p.ldsz = tile(g.Lz, p.Wz, p.Bz);
    p.ldst = tile(g.Lt, p.Wt, p.Bt);
    p.lds = std::max(p.ldsz, p.ldst);
    return p;
}

template <class T> void fft_set_max_lds(const geom &g, const zt_plan &p) {
    auto set = [](const void *f, size_t b) {
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
    };
    if (p.rc) {
#define LGF_ZTA(NN)                                                                 \
    case NN:                                                                        \
        set(reinterpret_cast<const void *>(&k_fft_zt_rc<T, NN, 0>), p.lds);        \
        set(reinterpret_cast<const void *>(&k_fft_zt_rc<T, NN, -1>), p.lds);       \
        set(reinterpret_cast<const void *>(&k_fft_zt_rc<T, NN, 1>), p.lds);        \
        break;
        switch (g.Lt) {
            LGF_NA_CASES(LGF_ZTA)
        default: break;
        }
#undef LGF_ZTA
    } else {
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 2, -1, 16>), p.ldsz);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 2, 1, 16>), p.ldsz);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 3, 0, 16>), p.ldst);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 3, -1, 16>), p.ldst);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 3, 1, 16>), p.ldst);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 2, -1, 32>), p.ldsz);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 2, 1, 32>), p.ldsz);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 3, 0, 32>), p.ldst);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 3, -1, 32>), p.ldst);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 3, 1, 32>), p.ldst);
    }
    if constexpr (std::is_same<T, float>::value) {
        if (!xy_use_rc<T>(g) && xy_acc_fusable<T>(g)) {
            const size_t b = xy_acc_lds_bytes<T>(g);
            set(reinterpret_cast<const void *>(&k_fft_xy_acc<T, 16, true>), b);
            set(reinterpret_cast<const void *>(&k_fft_xy_acc<T, 16, false>), b);
            set(reinterpret_cast<const void *>(&k_fft_xy_acc<T, 32, true>), b);
            set(reinterpret_cast<const void *>(&k_fft_xy_acc<T, 32, false>), b);
        }
    }
    if (!xy_use_rc<T>(g)) {
        const size_t b = fft_xy_lds_bytes<T>(g);
        set(reinterpret_cast<const void *>(&k_fft_xy<T, -1, 16>), b);
        set(reinterpret_cast<const void *>(&k_fft_xy<T, 1, 16>), b);
        set(reinterpret_cast<const void *>(&k_fft_xy<T, -1, 32>), b);
        set(reinterpret_cast<const void *>(&k_fft_xy<T, 1, 32>), b);
    }
}

template <class T>
hipError_t launch_fft_zt(const geom &g, void *D, int mode, const void *tw, const T *ptab,
                         T p2max_over_V, const zt_plan &pl, const dev_status *status,
                         hipStream_t st) {
    const long Lxy = (long)g.Lx * g.Ly;
    const int W = pl.W;
    dim3 grid((unsigned)((Lxy + W - 1) / W), (unsigned)g.nf);
    auto Dp = static_cast<vec2_t<T> *>(D);
    auto twp = static_cast<const vec2_t<T> *>(tw);
    if (pl.rc) {
        const unsigned nt = (unsigned)(W * g.Lz);
#define LGF_ZT(NN)                                                                                \
    case NN:                                                                                      \
        if (mode == 0)                                                                            \
            k_fft_zt_rc<T, NN, 0><<<grid, nt, pl.lds, st>>>(g, Dp, twp, ptab, p2max_over_V, W,   \
                                                            status);                              \
        else if (mode < 0)                                                                        \
            k_fft_zt_rc<T, NN, -1><<<grid, nt, pl.lds, st>>>(g, Dp, twp, ptab, p2max_over_V, W,  \
                                                             status);                             \
        else                                                                                      \
            k_fft_zt_rc<T, NN, 1><<<grid, nt, pl.lds, st>>>(g, Dp, twp, ptab, p2max_over_V, W,   \
                                                            status);                              \
        break;
        switch (g.Lt) {
            LGF_NA_CASES(LGF_ZT)
        default: return hipErrorInvalidValue;
        }
#undef LGF_ZT
        return hipGetLastError();
    }
    // z forward (mode <= 0), the t pass (forward, scaled round trip or
    // inverse), z inverse (mode >= 0); each axis takes the instance for its
    // extent's register span
    const unsigned nf = (unsigned)g.nf;
    const dim3 gz((unsigned)((Lxy + pl.Wz - 1) / pl.Wz), (unsigned)(g.Lt / pl.Bz), nf);
    const dim3 gt((unsigned)((Lxy + pl.Wt - 1) / pl.Wt), (unsigned)(g.Lz / pl.Bt), nf);
    const bool zs = fft_reg_span(g.Lz) <= 16, ts = fft_reg_span(g.Lt) <= 16;
    hipError_t e = hipSuccess;
    auto chk = [&] {
        if (e == hipSuccess) e = hipGetLastError();
    };
#define LGF_AXIS(AXN, MD, GRID, LDSB, WW, BB, SMALL)                                              \
    do {                                                                                          \
        if (SMALL)                                                                                \
            k_fft_axis<T, AXN, MD, 16><<<GRID, AXIS_BLOCK, LDSB, st>>>(g, Dp, twp, ptab,          \
                                                                      p2max_over_V, WW, BB,       \
                                                                      status);                    \
        else                                                                                      \
            k_fft_axis<T, AXN, MD, 32><<<GRID, AXIS_BLOCK, LDSB, st>>>(g, Dp, twp, ptab,          \
                                                                      p2max_over_V, WW, BB,       \
                                                                      status);                    \
        chk();                                                                                    \
    } while (0)
    if (mode <= 0) LGF_AXIS(2, -1, gz, pl.ldsz, pl.Wz, pl.Bz, zs);
    if (mode == 0) LGF_AXIS(3, 0, gt, pl.ldst, pl.Wt, pl.Bt, ts);
    else if (mode < 0) LGF_AXIS(3, -1, gt, pl.ldst, pl.Wt, pl.Bt, ts);
    else LGF_AXIS(3, 1, gt, pl.ldst, pl.Wt, pl.Bt, ts);
    if (mode >= 0) LGF_AXIS(2, 1, gz, pl.ldsz, pl.Wz, pl.Bz, zs);
#undef LGF_AXIS
    return e;
}

}  // namespace lgf
