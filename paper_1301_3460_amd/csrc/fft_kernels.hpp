// FFT pass kernels and their launchers, templated on the real type.  The
// translation units fft_f64.hip and fft_f32.hip instantiate them.
//
//   k_fft_xy_rc / k_fft_zt_rc  one axis held in registers, the other
//                              exchanged through LDS (extents <= 32)
//   k_fft_xy_rc2 / k_fft_zt_rc2  the same for FP64 32 x 32, two tiles per
//                              block (the second loaded during the first)
//   k_fft_xy                   a whole (x,y) plane in LDS (larger extents)
//   k_fft_tile2 (_acc)         two axes per pass in LDS: (x,t) planes and
//                              (y,z) tiles when (z,t) has an extent above 32
//   k_fft_axis                 one axis per pass: W inner sites x the axis x B
//                              slices in LDS (whatever the other schemes
//                              cannot hold)
//
// Twiddles: `tw` is the context's table buffer holding the axis tables of x,
// y, z and t one after the other (Lx, Ly, Lz and Lt entries); a transform
// along an axis reads only that axis's table.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace lgf {

static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

// Every listed extent is supported and every supported extent is listed.
#define LGF_COUNT_ONE(n) +1
#define LGF_AND_SUPPORTED(n) &&fft_supported(n)
constexpr int fft_count_supported() {
    int c = 0;
    for (int n = 2; n <= FFT_MAX_EXTENT; ++n)
        if (fft_supported(n)) ++c;
    return c;
}
static_assert(fft_count_supported() == 0 LGF_FFT_EXTENTS(LGF_COUNT_ONE), "extent list");
static_assert(true LGF_FFT_EXTENTS(LGF_AND_SUPPORTED), "extent list");
#undef LGF_COUNT_ONE
#undef LGF_AND_SUPPORTED

// axis tables inside the table buffer
template <class T> __host__ __device__ inline const vec2_t<T> *tw_y(const geom &g, const vec2_t<T> *tw) {
    return tw + g.Lx;
}
template <class T> __host__ __device__ inline const vec2_t<T> *tw_z(const geom &g, const vec2_t<T> *tw) {
    return tw + g.Lx + g.Ly;
}
template <class T> __host__ __device__ inline const vec2_t<T> *tw_t(const geom &g, const vec2_t<T> *tw) {
    return tw + g.Lx + g.Ly + g.Lz;
}

// Momentum-space factor p2max/(V p2) of one (z,t) column: `base` is the
// column's p2 without the z term (negative for a padding column).
template <class T>
__device__ __forceinline__ T fa_factor(T base, T pz, T p2max_over_V) {
    const T p2 = base + pz;
    return (base < T(0) || p2 == T(0)) ? T(0) : p2max_over_V * recip(p2);
}

// Element i = a + A (b + B c) of a tile as its digits (a, b, c), advanced by
// a fixed step with one carry per digit (the step's a and b digits are below
// A and B, so each sum stays below twice the radix).
struct tile_idx {
    int a, b, c;
    __device__ __forceinline__ tile_idx(int i, int A, int B) {
        a = i % A;
        const int r = i / A;
        b = r % B;
        c = r / B;
    }
    __device__ __forceinline__ void step(const tile_idx &d, int A, int B) {
        a += d.a;
        int k = a >= A;
        if (k) a -= A;
        b += d.b + k;
        k = b >= B;
        if (k) b -= B;
        c += d.c + k;
    }
};

// Copies the nel elements of a tile (digits a, b, c with radices A, B) from
// one memory to the other: each thread issues up to CH loads (get) before its
// first store (put), so that their latencies overlap (CH = 1: one round trip
// per element).
template <int NTHR, int CH, class V, class Get, class Put>
__device__ __forceinline__ void tile_copy(int nel, int A, int B, Get get, Put put) {
    const tile_idx d(NTHR, A, B);
    tile_idx q((int)threadIdx.x, A, B);
    for (int i0 = threadIdx.x; i0 < nel; i0 += CH * NTHR) {
        V v[CH];
        tile_idx p = q;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (i0 + k * NTHR < nel) v[k] = get(p);
            p.step(d, A, B);
        }
        p = q;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (i0 + k * NTHR < nel) put(p, v[k]);
            p.step(d, A, B);
        }
        q = p;
    }
}

// ---------------------------------------------------------------------------
// (x, y) plane transform: one plane of one field per block, LDS [y][x+1]
// ---------------------------------------------------------------------------

constexpr int XY_BLOCK = 256;
// a whole (x,y) plane of one field in LDS up to this size; larger planes take
// an x pass and a y pass
constexpr size_t XY_PLANE_LDS_MAX = 160 * 1024;

// RMAX: largest register tier (fft_tier) of the extents this instance handles
template <class T, int DIR, int RMAX>
__global__ void __launch_bounds__(XY_BLOCK)
    k_fft_xy(geom g, vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ tw,
             const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    const int Lx = g.Lx, Ly = g.Ly, P = Lx + 1;
    const long Lxy = (long)Lx * Ly;
    const vec2_t<T> *twx = tw, *twy = tw_y<T>(g, tw);
    vec2_t<T> *plane = D + (long)blockIdx.y * g.S + (long)blockIdx.x * Lxy;
    // Planes of at least four elements per thread keep nine loads per thread
    // in flight (plane digits x, y) and batch the stores of the forward pass,
    // as the (x,t) planes of k_fft_tile2 (64 x 64: 48 / 45 µs forward /
    // inverse against 53 / 46); smaller planes copy one element at a time
    // (8 x 64: 75 / 63 µs, against 79 / 67 through the batched copy).
    const bool batch = Lxy >= 4 * XY_BLOCK;
    if (batch) {
        tile_copy<XY_BLOCK, 9, vec2_t<T>>(
            (int)Lxy, Lx, Ly, [=](const tile_idx &p) { return plane[p.a + p.b * Lx]; },
            [=](const tile_idx &p, vec2_t<T> v) { lds[p.b * P + p.a] = v; });
    } else {
        for (int i = threadIdx.x; i < Lxy; i += XY_BLOCK) {
            const int y = i / Lx, x = i - y * Lx;
            lds[y * P + x] = plane[i];
        }
    }
    __syncthreads();
    auto rows = [P](int c) { return c * P; };
    auto cols = [](int c) { return c; };
    if (DIR < 0) {
        lds_axis_fft<DIR, T, RMAX>(Lx, lds, Ly, 1, rows, twx);
        __syncthreads();
        lds_axis_fft<DIR, T, RMAX>(Ly, lds, Lx, P, cols, twy);
    } else {
        lds_axis_fft<DIR, T, RMAX>(Ly, lds, Lx, P, cols, twy);
        __syncthreads();
        lds_axis_fft<DIR, T, RMAX>(Lx, lds, Ly, 1, rows, twx);
    }
    __syncthreads();
    if (batch && DIR < 0) {
        tile_copy<XY_BLOCK, 9, vec2_t<T>>(
            (int)Lxy, Lx, Ly, [=](const tile_idx &p) { return lds[p.b * P + p.a]; },
            [=](const tile_idx &p, vec2_t<T> v) { plane[p.a + p.b * Lx] = v; });
    } else {
        for (int i = threadIdx.x; i < Lxy; i += XY_BLOCK) {
            const int y = i / Lx, x = i - y * Lx;
            plane[i] = lds[y * P + x];
        }
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
    // digits (x, y, field), nine loads per thread in flight (64 x 64 planes:
    // 48 against 53 µs)
    tile_copy<XY_BLOCK, 9, vec2_t<T>>(
        4 * Lxy, Lx, Ly, [=](const tile_idx &p) { return D[(long)p.c * g.S + s0 + p.a + p.b * Lx]; },
        [=](const tile_idx &p, vec2_t<T> v) { lds[p.c * REG + p.b * P + p.a] = v; });
    __syncthreads();
    auto cols = [Lx, REG](int cc) { return (cc / Lx) * REG + (cc % Lx); };      // cc = x + Lx f
    auto rows = [Ly, REG, P](int cc) { return (cc / Ly) * REG + (cc % Ly) * P; };  // cc = y + Ly f
    lds_axis_fft<+1, T, RMAX>(Ly, lds, 4 * Lx, P, cols, tw_y<T>(g, tw));
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
// One-axis passes (axis_plan): for (z,t) planes too large for a register
// column (an extent above 32) the (z,t) transform becomes three passes over
// the field, z forward, then t forward / scaling / t inverse, then z inverse;
// (x,y) planes too large for LDS take an x pass and a y pass.  A block holds
// W inner elements (rows of up to 1 KB) x the whole axis x B slices, so every
// load and store is a contiguous row; the transform of each column runs in
// LDS (lds_axis_fft, one or two passes).
// MODE -1 forward, +1 inverse, 0 (t axis only) forward, times p2max/(V p2),
// inverse.
// ---------------------------------------------------------------------------

constexpr int AXIS_BLOCK = 256;
constexpr int ZT_PAD = 4;
// 32 KB tiles let four blocks share a compute unit (the register limit of
// these kernels); 64 KB tiles, with wider rows but three blocks, took 15-25%
// longer at 48^3 x 96.
constexpr size_t AXIS_TILE_BYTES = 32 * 1024;


// Register budgets: 128 VGPRs for tier 16 (four waves per SIMD, the
// occupancy the 32 KB tiles allow; the fused scaled round trip would take
// 129), 256 for tier 32 (without the hint it spills to AGPRs).
template <class T, int MODE, int RMAX>
__global__ void __launch_bounds__(AXIS_BLOCK) __attribute__((amdgpu_waves_per_eu(RMAX <= 16 ? 4 : 2)))
    k_fft_axis(geom g, vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ twa,
               const T *__restrict__ ptab, T p2max_over_V, axis_plan ap,
               const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    const int N = ap.N, W = ap.W, PW = ap.PW, PB = ap.PB;
    const long s0 = (long)xcd_block(blockIdx.x, gridDim.x) * W;
    const int Wt = (int)min((long)W, ap.R - s0);
    const int o0 = blockIdx.y * ap.B;  // first slice (B divides the slice count)
    vec2_t<T> *F = D + (long)blockIdx.z * g.S + s0 + (long)o0 * ap.sb;
    // offsets inside one field are below 2^31 (the volume is)
    const unsigned sj = (unsigned)ap.sj, sb = (unsigned)ap.sb;
    const int nel = W * N * ap.B;
    // tile digits (w, j, b), eight loads per thread in flight (the three
    // passes of 8 x 64^3: 173 against 193 µs in FP64, 96 against 107 in FP32);
    // a padding column of a ragged tile reads the tile's last column and
    // stores zero
    auto hbm = [=](int w, int j, int b) { return F + ((unsigned)j * sj + (unsigned)b * sb + (unsigned)w); };
    tile_copy<AXIS_BLOCK, 8, vec2_t<T>>(
        nel, W, N, [=](const tile_idx &p) { return *hbm(min(p.a, Wt - 1), p.b, p.c); },
        [=](const tile_idx &p, vec2_t<T> v) {
            if (p.a >= Wt) v.x = v.y = T(0);
            lds[p.c * PB + p.b * PW + p.a] = v;
        });
    __syncthreads();
    auto col = [W, PB](int c) { return (c / W) * PB + (c % W); };  // c = w + W*b
    if (MODE == 0) {
        // the t axis: inner elements are xy-sites, slices are z
        const T *px = ptab, *py = ptab + g.Lx, *pz = ptab + g.Lx + g.Ly,
                *pt = ptab + g.Lx + g.Ly + g.Lz;
        const long Lxy = (long)g.Lx * g.Ly;
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
        lds_axis_fsi<T, RMAX>(N, lds, W * ap.B, PW, col, prep, scale, twa);
    } else {
        lds_axis_fft<MODE, T, RMAX>(N, lds, W * ap.B, PW, col, twa);
    }
    __syncthreads();
    tile_copy<AXIS_BLOCK, 1, vec2_t<T>>(
        nel, W, N, [=](const tile_idx &p) { return lds[p.c * PB + p.b * PW + p.a]; },
        [=](const tile_idx &p, vec2_t<T> v) {
            if (p.a < Wt) *hbm(p.a, p.b, p.c) = v;
        });
}

// ---------------------------------------------------------------------------
// Two-axis LDS tiles (tile2_plan).  With an extent above 32 in (z,t) the
// transform is split as (x,t) planes and (y,z) tiles instead: the first and
// last passes hold whole (x,t) planes of one field (rows of Lx contiguous
// sites), the middle pass holds W consecutive x-sites x the (y,z) plane and
// runs the forward transforms, the scaling and the inverse transforms.  Three
// passes over the field instead of five.
// MODE -1: a forward then b forward; +1: b inverse then a inverse; 0: a
// forward, b forward / scaling / b inverse, a inverse.
// ---------------------------------------------------------------------------

// NTHR: threads per block; at the lighter register tier 512 where two tiles
// share a compute unit and 1024 where one tile fills it (16 waves either
// way), 256 at the wider tier
template <class T, int MODE, int RMAX, int NTHR>
__global__ void __launch_bounds__(NTHR)
    k_fft_tile2(geom g, vec2_t<T> *__restrict__ D, const vec2_t<T> *__restrict__ tw,
                const T *__restrict__ ptab, T p2max_over_V, tile2_plan tp,
                const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    // inner groups of one outer slice are consecutive on one XCD (they share lines)
    const int B = xcd_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int grp = B % tp.ngrp, outer = B / tp.ngrp;
    const int W = tp.W, Na = tp.Na, Nb = tp.Nb, PA = tp.PA, PB = tp.PB;
    const long i0 = (long)grp * W;
    const int Wt = (int)min((long)W, tp.R - i0);
    vec2_t<T> *F = D + (long)blockIdx.z * g.S + i0 + (long)outer * tp.so;
    // offsets inside one field are below 2^31 (the volume is)
    const unsigned sa = (unsigned)tp.sa, sb = (unsigned)tp.sb;
    const int nel = W * Na * Nb;
    // Loads per thread in flight in the copies, as measured at 48^3 x 96:
    // nine (0.33 against 0.41 ms in the FP64 first pass), three in the FP32
    // first pass (0.17 against 0.20), one in the FP64 middle pass, whose
    // 32-byte rows are shared by four blocks (0.68 ms; 0.94 with nine loads,
    // 0.73 with nine loads and nine stores, 0.92 with three of each).  Stores
    // are batched in the first pass only (the FP64 last pass: 0.34 ms with
    // single stores, 0.37 batched).
    constexpr int CHL = (MODE == 0 && sizeof(T) == 8) ? 1 : (MODE < 0 && sizeof(T) == 4) ? 3 : 9;
    constexpr int CHS = MODE < 0 ? CHL : 1;
    // tile digits (w, ja, jb); a padding column of a ragged group reads its
    // group's last column and stores zero
    auto hbm = [=](const tile_idx &p) { return F + ((unsigned)p.b * sa + (unsigned)p.c * sb + (unsigned)p.a); };
    auto sh = [=](const tile_idx &p) { return lds + (p.a + p.b * PA + p.c * PB); };
    tile_copy<NTHR, CHL, vec2_t<T>>(
        nel, W, Na,
        [=](const tile_idx &p) {
            tile_idx q = p;
            q.a = min(q.a, Wt - 1);
            return *hbm(q);
        },
        [=](const tile_idx &p, vec2_t<T> v) {
            if (p.a >= Wt) v.x = v.y = T(0);
            *sh(p) = v;
        });
    __syncthreads();
    const vec2_t<T> *twa = tw + tp.ta, *twb = tw + tp.tb;
    auto cola = [W, PB](int c) { return (c % W) + (c / W) * PB; };  // c = w + W*jb
    auto colb = [W, PA](int c) { return (c % W) + (c / W) * PA; };  // c = w + W*ja
    if (MODE <= 0) {
        lds_axis_fft<-1, T, RMAX>(Na, lds, W * Nb, PA, cola, twa);
        __syncthreads();
    }
    if (MODE == 0) {
        const T *pa = ptab + tp.ta, *pb = ptab + tp.tb, *pw = ptab + tp.tw, *po = ptab + tp.to;
        const long R = tp.R;
        // per column c = w + W*ja along b: p2 without the b term, or -1 for a
        // padding column of a ragged group (factor 0)
        auto prep = [=](int c) -> T {
            const int w = c % W, ja = c / W;
            if (i0 + w >= R) return T(-1);
            return (pa[ja] + pw[i0 + w]) + po[outer];
        };
        auto scale = [=](T base, int k) -> T { return fa_factor<T>(base, pb[k], p2max_over_V); };
        lds_axis_fsi<T, RMAX>(Nb, lds, W * Na, PB, colb, prep, scale, twb);
        __syncthreads();
    } else if (MODE < 0) {
        lds_axis_fft<-1, T, RMAX>(Nb, lds, W * Na, PB, colb, twb);
        __syncthreads();
    } else {
        lds_axis_fft<1, T, RMAX>(Nb, lds, W * Na, PB, colb, twb);
        __syncthreads();
    }
    if (MODE >= 0) {
        lds_axis_fft<1, T, RMAX>(Na, lds, W * Nb, PA, cola, twa);
        __syncthreads();
    }
    tile_copy<NTHR, CHS, vec2_t<T>>(
        nel, W, Na, [=](const tile_idx &p) { return *sh(p); },
        [=](const tile_idx &p, vec2_t<T> v) {
            if (p.a < Wt) *hbm(p) = v;
        });
}

// Last pass of the FP32 sweeps of an SU(3) mixed solve in the (x,t)/(y,z)
// split, fused with G(x) <- g(x) G(x): the (x,t) planes of all 4 fields of
// one (y,z) slice per block (4 LDS regions), inverse t and x transforms, then
// each site's 4 entries of L Delta form g and G goes from Gold into Gnew.
// L Delta itself is not stored.
// LDS of the 4-field planes of the fused inverse passes (one block per compute unit)
constexpr size_t XY_ACC_LDS_MAX = 150 * 1024;
// one block per compute unit: 16 waves at the lighter register tier, 8 at the other
template <int RMAX> constexpr int tile2_acc_threads() { return RMAX <= 16 ? 1024 : 512; }
template <int RMAX, bool EXACT>
__global__ void __launch_bounds__(tile2_acc_threads<RMAX>())
    k_fft_tile2_acc(geom g, const vec2_t<float> *__restrict__ D, const vec2_t<float> *__restrict__ tw,
                    const vec2_t<float> *__restrict__ Gold, vec2_t<float> *__restrict__ Gnew,
                    double c, tile2_plan tp, const dev_status *__restrict__ status) {
    using T = float;
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<T> *lds = reinterpret_cast<vec2_t<T> *>(smem_raw);
    const int Na = tp.Na, Nb = tp.Nb, PA = tp.PA, PB = tp.PB, REG = Nb * PB;
    const long off = (long)xcd_block(blockIdx.x, gridDim.x) * tp.so;
    const unsigned sb = (unsigned)tp.sb;  // the planes have one inner element (W = 1)
    const int nel = Na * Nb;
    // digits (ja, jb, field); nine loads per thread in flight (0.33 ms
    // against 0.38 at 48^3 x 96)
    tile_copy<tile2_acc_threads<RMAX>(), 9, vec2_t<T>>(
        4 * nel, Na, Nb,
        [=](const tile_idx &p) { return D[(long)p.c * g.S + off + (unsigned)p.a + (unsigned)p.b * sb]; },
        [=](const tile_idx &p, vec2_t<T> v) { lds[p.c * REG + p.a * PA + p.b * PB] = v; });
    __syncthreads();
    auto colb = [Na, PA, REG](int cc) { return (cc / Na) * REG + (cc % Na) * PA; };  // cc = ja + Na f
    auto cola = [Nb, PB, REG](int cc) { return (cc / Nb) * REG + (cc % Nb) * PB; };  // cc = jb + Nb f
    lds_axis_fft<1, T, RMAX>(Nb, lds, 4 * Na, PB, colb, tw + tp.tb);
    __syncthreads();
    lds_axis_fft<1, T, RMAX>(Na, lds, 4 * Nb, PA, cola, tw + tp.ta);
    __syncthreads();
    for (int i = threadIdx.x; i < nel; i += tile2_acc_threads<RMAX>()) {
        const int ja = i % Na, jb = i / Na;
        const vec2_t<T> *q = lds + ja * PA + jb * PB;
        accumulate_G<EXACT>(ld<T>(q), ld<T>(q + REG), ld<T>(q + 2 * REG), ld<T>(q + 3 * REG), c,
                            Gold, Gnew, g.S, off + (unsigned)ja + (unsigned)jb * sb);
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
        LGF_FFT_SMALL_EXTENTS(LGF_SCASE)
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
        LGF_FFT_SMALL_EXTENTS(LGF_CCASE)
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
    const vec2_t<T> *twy = tw_y<T>(g, tw);
    vec2_t<T> *p = D + (long)f * g.S + (long)blockIdx.x * Lxy + x;
    cpx<T> a[NY];
#pragma unroll
    for (int y = 0; y < NY; ++y) a[y] = ld<T>(p + (long)y * Lx);
    auto base = [F, SW, PJ](int c) { return (c / F) * PJ + (c % F) * SW; };  // c = fl + F*j
    auto col = [&](int, int C) { col_fft_small<DIR, T>(Lx, lds, F * C, 1, base, tw); };
    if (DIR < 0) {
        dft<NY, -1>(a, twy);
        exchange_axis<NY, T>(a, fl, x, 1, SW, PJ, lds, col);
    } else {
        exchange_axis<NY, T>(a, fl, x, 1, SW, PJ, lds, col);
        dft<NY, +1>(a, twy);
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
    dft<NY, +1>(a, tw_y<T>(g, tw));
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
    const vec2_t<T> *twz = tw_z<T>(g, tw), *twt = tw_t<T>(g, tw);
    vec2_t<T> *p = D + (long)blockIdx.y * g.S + (long)z * Lxy + s0 + w;
    const long tstride = (long)Lz * Lxy;
    cpx<T> a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = live ? ld<T>(p + t * tstride) : mk<T>(0, 0);
    const int PJ = Lz * W + ZT_PAD;
    auto base = [W, PJ](int c) { return (c / W) * PJ + (c % W); };  // c = w + W*j
    if (MODE <= 0) dft<NT, -1>(a, twt);
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
            col_fwd_scale_inv<T>(Lz, lds, W * C, W, base, prep, scale, twz);
        };
        exchange_axis<NT, T>(a, w, z, W, 1, PJ, lds, col);
    } else {
        auto col = [&](int, int C) { col_fft_small<MODE, T>(Lz, lds, W * C, W, base, twz); };
        exchange_axis<NT, T>(a, w, z, W, 1, PJ, lds, col);
    }
    if (MODE >= 0) dft<NT, +1>(a, twt);
    if (live) {
#pragma unroll
        for (int t = 0; t < NT; ++t) st<T>(p + t * tstride, a[t]);
    }
}

// ---------------------------------------------------------------------------
// Two-tile register-column passes (FP64, 32 x 32).
//
// A block of the kernels above moves one tile: it loads it, transforms it
// through LDS and stores it.  A 32-point FP64 column pins a wave to its SIMD
// alone (registers and LDS), and with two such rounds of blocks per compute
// unit the loads, the arithmetic and the stores of a round run one after the
// other.  Here a block takes tiles k and k + G (G blocks, half the tile
// count, so that every compute unit still holds two): the second tile's
// columns are loaded into registers (the accumulation registers take what
// does not fit) while the first tile goes through its LDS phase, inverse
// transform and stores.  The momentum table is copied into LDS, so the
// column phase issues no vector-memory load whose wait would also drain the
// prefetch.  Every tile goes through the same operations as in the one-tile
// kernels: the results are bitwise identical.
// ---------------------------------------------------------------------------

constexpr int RC2_N = 32;  // both register-column extents of the two-tile passes
constexpr int RC2_ZT_W = 4;  // xy-sites per (z,t) tile (64-byte rows)
constexpr int RC2_XY_F = 4;  // fields per (x,y) tile (all of an SU(3) plane)

template <int N>
__device__ __forceinline__ void load_column(const double2 *p, unsigned stride,
                                            cpx<double> (&a)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] = ld<double>(p + j * stride);
}

template <int N>
__device__ __forceinline__ void store_column(double2 *p, unsigned stride, const cpx<double> (&a)[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) st<double>(p + j * stride, a[j]);
}

// (z,t): tile k = W consecutive xy-sites of field k / (Lxy / W); thread
// (w, z) holds the t-column of site s0 + w at z.  MODE 0 only.
template <int NZ, int NT, int W, class Hook>
__device__ __forceinline__ void zt2_tile(const geom &g, int s0, cpx<double> (&a)[NT], Hook prefetch,
                                         vec2_t<double> *lds, const vec2_t<double> *twz,
                                         const vec2_t<double> *twt, const double *pz,
                                         double p2max_over_V) {
    using T = double;
    constexpr int PJ = NZ * W + ZT_PAD;
    const int w = threadIdx.x % W, z = threadIdx.x / W;
    const T *q = reinterpret_cast<const T *>(lds + NT * PJ);
    const T *qx = q, *qy = q + g.Lx, *qt = q + g.Lx + g.Ly + NZ;
    const int Lx = g.Lx;
    auto base = [](int c) { return (c / W) * PJ + (c % W); };  // c = w + W*j
    dft<NT, -1>(a, twt);
    auto col = [&](int c0, int C) {
        auto prep = [=](int c) -> T {
            const int sxy = s0 + (c % W);  // the tiles are whole
            const int y = sxy / Lx, x = sxy - y * Lx;
            return (qx[x] + qy[y]) + qt[c0 + c / W];
        };
        auto scale = [=](T b, int k) -> T { return fa_factor<T>(b, pz[k], p2max_over_V); };
        prefetch();
        col_fwd_scale_inv_n<NZ, T>(lds, W * C, W, base, prep, scale, twz);
    };
    exchange_axis<NT, T>(a, w, z, W, 1, PJ, lds, col);
    dft<NT, +1>(a, twt);
}

template <int NZ, int NT, int W>
__global__ void __launch_bounds__(NZ * W) __attribute__((amdgpu_waves_per_eu(1, 1)))
    k_fft_zt_rc2(geom g, vec2_t<double> *__restrict__ D, const vec2_t<double> *__restrict__ tw,
                 const double *__restrict__ ptab, double p2max_over_V,
                 const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<double> *lds = reinterpret_cast<vec2_t<double> *>(smem_raw);
    {
        double *q = reinterpret_cast<double *>(lds + NT * (NZ * W + ZT_PAD));
        const int n = g.Lx + g.Ly + NZ + NT;
        for (int i = threadIdx.x; i < n; i += NZ * W) q[i] = ptab[i];
    }
    const unsigned Lxy = (unsigned)g.Lx * (unsigned)g.Ly, ts = (unsigned)NZ * Lxy;
    const int ntx = (int)(Lxy / W), G = gridDim.x;
    const int w = threadIdx.x % W, z = threadIdx.x / W;
    const int k0 = xcd_block(blockIdx.x, G), k1 = k0 + G;
    const int f0 = k0 / ntx, f1 = k1 / ntx;
    const int s0 = (k0 - f0 * ntx) * W, s1 = (k1 - f1 * ntx) * W;
    vec2_t<double> *p0 = D + (long)f0 * g.S + (unsigned)z * Lxy + (unsigned)(s0 + w);
    vec2_t<double> *p1 = D + (long)f1 * g.S + (unsigned)z * Lxy + (unsigned)(s1 + w);
    const vec2_t<double> *twz = tw_z<double>(g, tw), *twt = tw_t<double>(g, tw);
    const double *pz = ptab + g.Lx + g.Ly;
    cpx<double> a[NT], b[NT];
    load_column<NT>(p0, ts, a);
    zt2_tile<NZ, NT, W>(g, s0, a, [&] { load_column<NT>(p1, ts, b); }, lds, twz, twt, pz,
                        p2max_over_V);
    __syncthreads();  // every thread has read its column of the first tile back
    store_column<NT>(p0, ts, a);
    zt2_tile<NZ, NT, W>(g, s1, b, [] {}, lds, twz, twt, pz, p2max_over_V);
    store_column<NT>(p1, ts, b);
}

// (x,y): tile k = plane k of all F fields; thread (f, x) holds a y-column.
template <int NX, int NY, int F, int DIR, class Hook>
__device__ __forceinline__ void xy2_tile(cpx<double> (&a)[NY], Hook prefetch, vec2_t<double> *lds,
                                         const vec2_t<double> *twx, const vec2_t<double> *twy) {
    using T = double;
    constexpr int SW = NX + 1, PJ = F * SW;
    const int x = threadIdx.x % NX, fl = threadIdx.x / NX;
    auto base = [](int c) { return (c / F) * PJ + (c % F) * SW; };  // c = fl + F*j
    auto col = [&](int, int C) {
        prefetch();
        lds_axis_fft_n<NX, DIR, T>(lds, F * C, 1, base, twx);
    };
    if (DIR < 0) {
        dft<NY, -1>(a, twy);
        exchange_axis<NY, T>(a, fl, x, 1, SW, PJ, lds, col);
    } else {
        exchange_axis<NY, T>(a, fl, x, 1, SW, PJ, lds, col);
        dft<NY, +1>(a, twy);
    }
}

template <int NX, int NY, int F, int DIR>
__global__ void __launch_bounds__(NX * F) __attribute__((amdgpu_waves_per_eu(1, 1)))
    k_fft_xy_rc2(geom g, vec2_t<double> *__restrict__ D, const vec2_t<double> *__restrict__ tw,
                 const dev_status *__restrict__ status) {
    if (status->done) return;
    extern __shared__ unsigned char smem_raw[];
    vec2_t<double> *lds = reinterpret_cast<vec2_t<double> *>(smem_raw);
    const int x = threadIdx.x % NX, fl = threadIdx.x / NX;
    const int k0 = blockIdx.x, k1 = k0 + gridDim.x;
    constexpr unsigned Lxy = (unsigned)NX * NY;
    vec2_t<double> *p0 = D + (long)fl * g.S + (unsigned)k0 * Lxy + x;
    vec2_t<double> *p1 = D + (long)fl * g.S + (unsigned)k1 * Lxy + x;
    const vec2_t<double> *twy = tw_y<double>(g, tw);
    cpx<double> a[NY], b[NY];
    load_column<NY>(p0, NX, a);
    xy2_tile<NX, NY, F, DIR>(a, [&] { load_column<NY>(p1, NX, b); }, lds, tw, twy);
    __syncthreads();  // every thread has read its column of the first tile back
    store_column<NY>(p0, NX, a);
    xy2_tile<NX, NY, F, DIR>(b, [] {}, lds, tw, twy);
    store_column<NY>(p1, NX, b);
}

// ---------------------------------------------------------------------------
// planning and launchers
// ---------------------------------------------------------------------------

template <class T> inline int xy_fields_per_block(const geom &g) {
    int F = g.nf;
    while (F > 1 && F * g.Lx > rc_max_threads<T>()) F >>= 1;
    return F;
}

// A one-axis pass over axis ax: rows of up to 1 KB (W consecutive inner
// elements; one element for the x axis), then as many slices as keep a tile
// within AXIS_TILE_BYTES.
template <class T> axis_plan plan_axis(const geom &g, int ax) {
    const int L[4] = {g.Lx, g.Ly, g.Lz, g.Lt};
    const long Lxy = (long)g.Lx * g.Ly;
    axis_plan a;
    a.N = L[ax];
    if (ax == 0) {
        a.R = 1;
        a.sj = 1;
        a.sb = g.Lx;
        a.nslice = g.Ly * g.Lz * g.Lt;
    } else if (ax == 1) {
        a.R = g.Lx;
        a.sj = g.Lx;
        a.sb = Lxy;
        a.nslice = g.Lz * g.Lt;
    } else if (ax == 2) {
        a.R = Lxy;
        a.sj = Lxy;
        a.sb = Lxy * g.Lz;
        a.nslice = g.Lt;
    } else {  // t: inner xy-sites, slices along z
        a.R = Lxy;
        a.sj = Lxy * g.Lz;
        a.sb = Lxy;
        a.nslice = g.Lz;
    }
    const size_t e = sizeof(vec2_t<T>);
    auto strides = [&](int w, int b, int &pw, int &pb) {
        pw = w == 1 ? 1 : w + 1;
        pb = a.N * pw;
        if (w == 1 && pb % 2 == 0) ++pb;  // columns of consecutive threads on odd strides
        return (size_t)b * pb * e;
    };
    int pw, pb;
    int w = (int)(1024 / e);
    while (w > 1 && (w > a.R || strides(w, 1, pw, pb) > AXIS_TILE_BYTES)) w >>= 1;
    // slices: a power of two dividing the slice count, at most 8 with rows
    // (64 for the x axis, whose rows are single elements)
    int b = a.R == 1 ? 64 : 8;
    while (b > 1 && (strides(w, b, pw, pb) > AXIS_TILE_BYTES || a.nslice % b != 0)) b >>= 1;
    a.W = w;
    a.B = b;
    a.lds = strides(w, b, pw, pb);
    a.PW = pw;
    a.PB = pb;
    return a;
}

// Two-tile passes: FP64, both extents 32, whole tiles, an even tile count
// of at least four per compute unit.
template <class T> void plan_two_tile(const geom &g, int ncu, fft_plan &p) {
    if (!std::is_same<T, double>::value || ncu <= 0) return;
    const long Lxy = (long)g.Lx * g.Ly;
    auto enough = [&](long tiles) { return tiles % 2 == 0 && tiles / 2 >= 2L * ncu; };
    p.xy2 = p.xy == 0 && g.Lx == RC2_N && g.Ly == RC2_N && g.nf == RC2_XY_F &&
            xy_fields_per_block<T>(g) == RC2_XY_F && enough((long)g.Lz * g.Lt);
    p.zt2 = p.rc && g.Lz == RC2_N && g.Lt == RC2_N && p.W == RC2_ZT_W && Lxy % RC2_ZT_W == 0 &&
            enough(Lxy / RC2_ZT_W * g.nf);
    if (p.zt2)
        p.lds_zt2 = p.lds + (size_t)(g.Lx + g.Ly + g.Lz + g.Lt) * sizeof(T);
}

// (x,t) planes and (y,z) tiles of 32-byte rows (2 FP64 or 4 FP32 x-sites),
// for an extent above 32 in (z,t), where both tiles fit and the planes' rows
// are at least 16 sites.
template <class T> void plan_tile2(const geom &g, size_t budget, fft_plan &p) {
    if (p.rc) return;
    constexpr int TILE2_W = 32 / (int)sizeof(vec2_t<T>);
    const size_t e = sizeof(vec2_t<T>);
    const long Lxy = (long)g.Lx * g.Ly, Lxyz = Lxy * g.Lz;
    const int ox = 0, oy = g.Lx, oz = g.Lx + g.Ly, ot = g.Lx + g.Ly + g.Lz;
    tile2_plan a;  // (x,t) planes: a = x (the rows), b = t; slices (y,z)
    a.Na = g.Lx;
    a.Nb = g.Lt;
    a.W = 1;
    a.sa = 1;
    a.sb = Lxyz;
    a.R = 1;
    a.ngrp = 1;
    a.nouter = g.Ly * g.Lz;
    a.so = g.Lx;
    a.PA = 1;
    a.PB = g.Lx + 1;
    a.ta = ox;
    a.tb = ot;
    a.rmax = std::max(fft_tier(g.Lx), fft_tier(g.Lt));
    a.lds = (size_t)a.Nb * a.PB * e;
    a.nthr = a.lds > 80 * 1024 ? 1024 : 512;
    tile2_plan b;  // (y,z) tiles: W x-sites, a = y, b = z; slices t
    b.Na = g.Ly;
    b.Nb = g.Lz;
    b.W = TILE2_W;
    b.sa = g.Lx;
    b.sb = Lxy;
    b.R = g.Lx;
    b.ngrp = (g.Lx + TILE2_W - 1) / TILE2_W;
    b.nouter = g.Lt;
    b.so = Lxyz;
    b.PA = TILE2_W;
    b.PB = g.Ly * TILE2_W + 1;
    b.ta = oy;
    b.tb = oz;
    b.tw = ox;
    b.to = ot;
    b.rmax = std::max(fft_tier(g.Ly), fft_tier(g.Lz));
    b.lds = (size_t)b.Nb * b.PB * e;
    b.nthr = b.lds > 80 * 1024 ? 1024 : 512;
    if (g.Lx < 16 || a.lds > budget || b.lds > 160 * 1024 || a.nouter > 65535) return;
    p.t2 = true;
    p.xy2 = false;  // the (x,t) planes replace the (x,y) pass
    p.t2a = a;
    p.t2b = b;
}

template <class T> fft_plan plan_fft(const geom &g, size_t zt_lds_budget, int ncu) {
    fft_plan p{};
    const size_t e = sizeof(vec2_t<T>);
    if (g.Lx <= 32 && g.Ly <= 32) {
        p.xy = 0;
        p.lds_xy = (size_t)g.Ly * xy_fields_per_block<T>(g) * (g.Lx + 1) * e;
    } else if ((size_t)g.Ly * (g.Lx + 1) * e <= XY_PLANE_LDS_MAX) {
        p.xy = 1;
        p.lds_xy = (size_t)g.Ly * (g.Lx + 1) * e;
    } else {
        p.xy = 2;
        p.x = plan_axis<T>(g, 0);
        p.y = plan_axis<T>(g, 1);
    }
    // (z,t): register-column kernel when both extents are at most 32 (tile of
    // W sites with 128-byte rows), else the z and t passes
    const long Lxy = (long)g.Lx * g.Ly;
    if (g.Lt <= 32 && g.Lz <= 32) {
        auto rc_bytes = [&](int w) { return (size_t)g.Lt * ((size_t)g.Lz * w + ZT_PAD) * e; };
        int W = 128 / (int)e;
        while (W > 1 && (W * g.Lz > rc_max_threads<T>() || W > Lxy || rc_bytes(W) > zt_lds_budget))
            W >>= 1;
        if (W * g.Lz <= rc_max_threads<T>() && rc_bytes(W) <= 160 * 1024) {
            p.rc = true;
            p.W = W;
            p.lds = rc_bytes(W);
            plan_two_tile<T>(g, ncu, p);
            return p;
        }
    }
    p.rc = false;
    p.z = plan_axis<T>(g, 2);
    p.t = plan_axis<T>(g, 3);
    p.W = p.z.W;
    p.lds = std::max(p.z.lds, p.t.lds);
    plan_two_tile<T>(g, ncu, p);
    plan_tile2<T>(g, zt_lds_budget, p);
    return p;
}

inline dim3 tile2_grid(const tile2_plan &a, int nf) {
    return dim3((unsigned)a.ngrp, (unsigned)a.nouter, (unsigned)nf);
}

template <class T, int MODE>
hipError_t launch_tile2(const geom &g, vec2_t<T> *D, const vec2_t<T> *tw, const T *ptab,
                        T p2max_over_V, const tile2_plan &a, const dev_status *status,
                        hipStream_t st) {
    const dim3 grid = tile2_grid(a, g.nf);
#define LGF_T2(R, N)                                                                               \
    k_fft_tile2<T, MODE, R, N><<<grid, N, a.lds, st>>>(g, D, tw, ptab, p2max_over_V, a, status)
    if (a.rmax > 16) LGF_T2(32, 256);
    else if (a.nthr == 1024) LGF_T2(16, 1024);
    else LGF_T2(16, 512);
#undef LGF_T2
    return hipGetLastError();
}

inline dim3 axis_grid(const axis_plan &a, int nf) {
    return dim3(nblk(a.R, a.W), nblk(a.nslice, a.B), (unsigned)nf);
}

template <class T> void fft_set_max_lds(const geom &g, const fft_plan &p) {
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
            LGF_FFT_SMALL_EXTENTS(LGF_ZTA)
        default: break;
        }
#undef LGF_ZTA
    }
    size_t ax = 0;
    if (!p.rc) ax = std::max(p.z.lds, p.t.lds);
    if (p.xy == 2) ax = std::max(ax, std::max(p.x.lds, p.y.lds));
    if (ax > 0) {
        set(reinterpret_cast<const void *>(&k_fft_axis<T, -1, 16>), ax);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 1, 16>), ax);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 0, 16>), ax);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, -1, 32>), ax);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 1, 32>), ax);
        set(reinterpret_cast<const void *>(&k_fft_axis<T, 0, 32>), ax);
    }
    if constexpr (std::is_same<T, float>::value) {
        if (p.xy == 1 && xy_acc_fusable<T>(g, p)) {
            const size_t b = (size_t)4 * g.Ly * (g.Lx + 1) * sizeof(vec2_t<T>);
            set(reinterpret_cast<const void *>(&k_fft_xy_acc<T, 16, true>), b);
            set(reinterpret_cast<const void *>(&k_fft_xy_acc<T, 16, false>), b);
            set(reinterpret_cast<const void *>(&k_fft_xy_acc<T, 32, true>), b);
            set(reinterpret_cast<const void *>(&k_fft_xy_acc<T, 32, false>), b);
        }
    }
    if (p.t2) {
        const size_t b = std::max(p.t2a.lds, p.t2b.lds);
#define LGF_T2S(M)                                                                   \
    set(reinterpret_cast<const void *>(&k_fft_tile2<T, M, 16, 512>), b);            \
    set(reinterpret_cast<const void *>(&k_fft_tile2<T, M, 16, 1024>), b);           \
    set(reinterpret_cast<const void *>(&k_fft_tile2<T, M, 32, 256>), b);
        LGF_T2S(-1) LGF_T2S(0) LGF_T2S(1)
#undef LGF_T2S
        if constexpr (std::is_same<T, float>::value) {
            const size_t a4 = 4 * p.t2a.lds;
            if (a4 <= XY_ACC_LDS_MAX) {
                set(reinterpret_cast<const void *>(&k_fft_tile2_acc<16, true>), a4);
                set(reinterpret_cast<const void *>(&k_fft_tile2_acc<16, false>), a4);
                set(reinterpret_cast<const void *>(&k_fft_tile2_acc<32, true>), a4);
                set(reinterpret_cast<const void *>(&k_fft_tile2_acc<32, false>), a4);
            }
        }
    }
    if constexpr (std::is_same<T, double>::value) {
        if (p.xy2) {
            set(reinterpret_cast<const void *>(&k_fft_xy_rc2<RC2_N, RC2_N, RC2_XY_F, -1>), p.lds_xy);
            set(reinterpret_cast<const void *>(&k_fft_xy_rc2<RC2_N, RC2_N, RC2_XY_F, 1>), p.lds_xy);
        }
        if (p.zt2)
            set(reinterpret_cast<const void *>(&k_fft_zt_rc2<RC2_N, RC2_N, RC2_ZT_W>), p.lds_zt2);
    }
    if (p.xy == 1) {
        set(reinterpret_cast<const void *>(&k_fft_xy<T, -1, 16>), p.lds_xy);
        set(reinterpret_cast<const void *>(&k_fft_xy<T, 1, 16>), p.lds_xy);
        set(reinterpret_cast<const void *>(&k_fft_xy<T, -1, 32>), p.lds_xy);
        set(reinterpret_cast<const void *>(&k_fft_xy<T, 1, 32>), p.lds_xy);
    }
}

// One one-axis pass (the instance for the axis extent's register span).
template <class T, int MODE>
hipError_t launch_axis(const geom &g, vec2_t<T> *D, const vec2_t<T> *twa, const T *ptab,
                       T p2max_over_V, const axis_plan &a, const dev_status *status,
                       hipStream_t st) {
    const dim3 grid = axis_grid(a, g.nf);
    if (fft_tier(a.N) <= 16)
        k_fft_axis<T, MODE, 16><<<grid, AXIS_BLOCK, a.lds, st>>>(g, D, twa, ptab, p2max_over_V, a,
                                                                 status);
    else
        k_fft_axis<T, MODE, 32><<<grid, AXIS_BLOCK, a.lds, st>>>(g, D, twa, ptab, p2max_over_V, a,
                                                                 status);
    return hipGetLastError();
}

template <class T>
hipError_t launch_fft_xy(const geom &g, void *D, int dir, const void *tw, const fft_plan &pl,
                         const dev_status *status, hipStream_t st) {
    auto Dp = static_cast<vec2_t<T> *>(D);
    auto twp = static_cast<const vec2_t<T> *>(tw);
    if (pl.t2) {
        // (x,t) planes: forward first, inverse last
        if (dir < 0) return launch_tile2<T, -1>(g, Dp, twp, nullptr, T(0), pl.t2a, status, st);
        return launch_tile2<T, 1>(g, Dp, twp, nullptr, T(0), pl.t2a, status, st);
    }
    if constexpr (std::is_same<T, double>::value) {
        if (pl.xy2) {
            const unsigned G = (unsigned)(g.Lz * g.Lt / 2);
            constexpr unsigned nt = RC2_N * RC2_XY_F;
            if (dir < 0)
                k_fft_xy_rc2<RC2_N, RC2_N, RC2_XY_F, -1><<<G, nt, pl.lds_xy, st>>>(g, Dp, twp, status);
            else
                k_fft_xy_rc2<RC2_N, RC2_N, RC2_XY_F, 1><<<G, nt, pl.lds_xy, st>>>(g, Dp, twp, status);
            return hipGetLastError();
        }
    }
    if (pl.xy == 0) {
        const int F = xy_fields_per_block<T>(g);
        dim3 grid((unsigned)(g.Lz * g.Lt), (unsigned)(g.nf / F));
        const unsigned nt = (unsigned)(F * g.Lx);
        const size_t lds = pl.lds_xy;
#define LGF_XY(NN)                                                                            \
    case NN:                                                                                  \
        if (dir < 0) k_fft_xy_rc<T, NN, -1><<<grid, nt, lds, st>>>(g, Dp, twp, F, status);   \
        else k_fft_xy_rc<T, NN, 1><<<grid, nt, lds, st>>>(g, Dp, twp, F, status);            \
        break;
        switch (g.Ly) {
            LGF_FFT_SMALL_EXTENTS(LGF_XY)
        default: return hipErrorInvalidValue;
        }
#undef LGF_XY
        return hipGetLastError();
    }
    if (pl.xy == 2) {
        // separate passes: x then y forward, y then x inverse
        hipError_t e;
        const T zero = T(0);
        if (dir < 0) {
            if ((e = launch_axis<T, -1>(g, Dp, twp, nullptr, zero, pl.x, status, st))) return e;
            return launch_axis<T, -1>(g, Dp, tw_y<T>(g, twp), nullptr, zero, pl.y, status, st);
        }
        if ((e = launch_axis<T, 1>(g, Dp, tw_y<T>(g, twp), nullptr, zero, pl.y, status, st)))
            return e;
        return launch_axis<T, 1>(g, Dp, twp, nullptr, zero, pl.x, status, st);
    }
    dim3 grid((unsigned)(g.Lz * g.Lt), (unsigned)g.nf);
    if (fft_tier(g.Lx) <= 16 && fft_tier(g.Ly) <= 16) {
        if (dir < 0) k_fft_xy<T, -1, 16><<<grid, XY_BLOCK, pl.lds_xy, st>>>(g, Dp, twp, status);
        else k_fft_xy<T, +1, 16><<<grid, XY_BLOCK, pl.lds_xy, st>>>(g, Dp, twp, status);
    } else {
        if (dir < 0) k_fft_xy<T, -1, 32><<<grid, XY_BLOCK, pl.lds_xy, st>>>(g, Dp, twp, status);
        else k_fft_xy<T, +1, 32><<<grid, XY_BLOCK, pl.lds_xy, st>>>(g, Dp, twp, status);
    }
    return hipGetLastError();
}

// The fused inverse pass with G accumulation: register-column planes
// holding all 4 fields in one block, or whole (x,y) or (x,t) planes of all 4
// fields in LDS.
template <class T> inline size_t xy_acc_lds_bytes(const geom &g) {
    return (size_t)4 * g.Ly * (g.Lx + 1) * sizeof(vec2_t<T>);
}
template <class T> bool xy_acc_fusable(const geom &g, const fft_plan &pl) {
    if (g.nc != 3 || g.nf != 4) return false;
    if (pl.t2) return std::is_same<T, float>::value && 4 * pl.t2a.lds <= XY_ACC_LDS_MAX;
    if (pl.xy == 0) return xy_fields_per_block<T>(g) == 4;
    if (pl.xy == 1) return xy_acc_lds_bytes<T>(g) <= XY_ACC_LDS_MAX;
    return false;
}

template <class T>
hipError_t launch_fft_xy_inv_acc(const geom &g, void *D, const void *tw, const fft_plan &pl,
                                 const void *Gold, void *Gnew, double c, bool exact,
                                 const dev_status *status, hipStream_t st) {
    if (!xy_acc_fusable<T>(g, pl)) return hipErrorInvalidValue;
    auto Dp = static_cast<const vec2_t<T> *>(D);
    auto twp = static_cast<const vec2_t<T> *>(tw);
    auto Go = static_cast<const vec2_t<T> *>(Gold);
    auto Gn = static_cast<vec2_t<T> *>(Gnew);
    if constexpr (std::is_same<T, float>::value) {
        if (pl.t2) {
            const dim3 grid((unsigned)pl.t2a.nouter);
            const size_t b = 4 * pl.t2a.lds;
#define LGF_TA(R, E)                                                                          \
    k_fft_tile2_acc<R, E><<<grid, tile2_acc_threads<R>(), b, st>>>(g, Dp, twp, Go, Gn, c, pl.t2a, \
                                                                  status)
            if (pl.t2a.rmax <= 16) {
                if (exact) LGF_TA(16, true);
                else LGF_TA(16, false);
            } else {
                if (exact) LGF_TA(32, true);
                else LGF_TA(32, false);
            }
#undef LGF_TA
            return hipGetLastError();
        }
    }
    if (pl.xy == 1) {
        const size_t b = xy_acc_lds_bytes<T>(g);
        const dim3 grid((unsigned)(g.Lz * g.Lt));
        const bool sm = fft_tier(g.Lx) <= 16 && fft_tier(g.Ly) <= 16;
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
    const size_t lds = pl.lds_xy;
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
        LGF_FFT_SMALL_EXTENTS(LGF_XA)
    default: return hipErrorInvalidValue;
    }
#undef LGF_XA
    return hipGetLastError();
}

template <class T>
hipError_t launch_fft_zt(const geom &g, void *D, int mode, const void *tw, const T *ptab,
                         T p2max_over_V, const fft_plan &pl, const dev_status *status,
                         hipStream_t st) {
    const long Lxy = (long)g.Lx * g.Ly;
    auto Dp = static_cast<vec2_t<T> *>(D);
    auto twp = static_cast<const vec2_t<T> *>(tw);
    if constexpr (std::is_same<T, double>::value) {
        if (pl.zt2 && mode == 0) {
            const unsigned G = (unsigned)(Lxy / RC2_ZT_W * g.nf / 2);
            k_fft_zt_rc2<RC2_N, RC2_N, RC2_ZT_W><<<G, RC2_N * RC2_ZT_W, pl.lds_zt2, st>>>(
                g, Dp, twp, ptab, p2max_over_V, status);
            return hipGetLastError();
        }
    }
    if (pl.t2) {
        // (y,z) tiles: forward, scaled round trip or inverse
        if (mode == 0) return launch_tile2<T, 0>(g, Dp, twp, ptab, p2max_over_V, pl.t2b, status, st);
        if (mode < 0) return launch_tile2<T, -1>(g, Dp, twp, ptab, p2max_over_V, pl.t2b, status, st);
        return launch_tile2<T, 1>(g, Dp, twp, ptab, p2max_over_V, pl.t2b, status, st);
    }
    if (pl.rc) {
        const int W = pl.W;
        dim3 grid((unsigned)((Lxy + W - 1) / W), (unsigned)g.nf);
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
            LGF_FFT_SMALL_EXTENTS(LGF_ZT)
        default: return hipErrorInvalidValue;
        }
#undef LGF_ZT
        return hipGetLastError();
    }
    // z forward (mode <= 0), the t pass (forward, scaled round trip or
    // inverse), z inverse (mode >= 0)
    const vec2_t<T> *twz = tw_z<T>(g, twp), *twt = tw_t<T>(g, twp);
    hipError_t e;
    if (mode <= 0 && (e = launch_axis<T, -1>(g, Dp, twz, ptab, p2max_over_V, pl.z, status, st)))
        return e;
    if (mode == 0) e = launch_axis<T, 0>(g, Dp, twt, ptab, p2max_over_V, pl.t, status, st);
    else if (mode < 0) e = launch_axis<T, -1>(g, Dp, twt, ptab, p2max_over_V, pl.t, status, st);
    else e = launch_axis<T, 1>(g, Dp, twt, ptab, p2max_over_V, pl.t, status, st);
    if (e) return e;
    if (mode >= 0) return launch_axis<T, 1>(g, Dp, twz, ptab, p2max_over_V, pl.z, status, st);
    return hipSuccess;
}

}  // namespace lgf
