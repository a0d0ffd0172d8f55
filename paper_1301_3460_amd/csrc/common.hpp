// Device helpers shared by the kernel translation units.
#pragma once
#include "fft.hpp"
#include "kernels.hpp"
#include "su3.hpp"

namespace lgf {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Blocks are dispatched round-robin over the 8 XCDs; map them so that each
// XCD (own L2) walks a contiguous range of sites and neighbour data is shared.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Site of thread tid of site-kernel block b.  Blocks are first remapped so
// that each XCD walks a contiguous range.
//   g.tblock == 0: consecutive sites.
//   g.tblock == 1: the block's four waves take 64 consecutive xy-sites (a
//     "segment", one coalesced row each) at 4 consecutive t.  Blocks advance
//     through a group of g.sgroup adjacent segments fastest, then z, then the
//     segment group, then t: three of four t-neighbour pairs are inside a
//     block, and the blocks holding the y and z neighbours are at most
//     g.sgroup positions apart in dispatch order on the same XCD, so their
//     lines are still in that XCD's L2.  When each XCD's range holds
//     g.tslab > 1 slices of 4 t, the slices are walked inside z (after the
//     segment group), so the t neighbours across two slices of one XCD are
//     g.sgroup positions apart too instead of a whole slice.
__device__ __forceinline__ long block_site(const geom &g, int b, int nb, int tid) {
    const int B = xcd_block(b, nb);
    if (!g.tblock) return (long)B * SITE_BLOCK + tid;
    const int Lxy = g.Lx * g.Ly, G = g.sgroup, ngrp = (Lxy >> 6) / G;
    const int sg = B % G;
    int r = B / G;
    const int sl = r % g.tslab;
    r /= g.tslab;
    const int z = r % g.Lz;
    r /= g.Lz;
    const int slab = (r / ngrp) * g.tslab + sl;
    const int seg = (r % ngrp) * G + sg, t = slab * 4 + (tid >> 6);
    return (long)seg * 64 + (tid & 63) + (long)Lxy * (z + (long)g.Lz * t);
}

struct nbr {
    long p[4], m[4];  // s + mu, s - mu (periodic)
};

// Site coordinates in 32-bit unsigned arithmetic (every supported volume,
// up to 128^4 sites, is below 2^31).
__device__ __forceinline__ nbr neighbours(const geom &g, long s) {
    nbr n;
    unsigned r = (unsigned)s;
    const unsigned Lx = g.Lx, Ly = g.Ly, Lz = g.Lz;
    unsigned q = r / Lx;
    const int x = (int)(r - q * Lx);
    r = q; q = r / Ly;
    const int y = (int)(r - q * Ly);
    r = q; q = r / Lz;
    const int z = (int)(r - q * Lz);
    const int t = (int)q;
    const long sy = g.Lx, sz = (long)g.Lx * g.Ly, stt = sz * g.Lz;
    n.p[0] = (x == g.Lx - 1) ? s - (g.Lx - 1) : s + 1;
    n.m[0] = (x == 0) ? s + (g.Lx - 1) : s - 1;
    n.p[1] = (y == g.Ly - 1) ? s - (long)(g.Ly - 1) * sy : s + sy;
    n.m[1] = (y == 0) ? s + (long)(g.Ly - 1) * sy : s - sy;
    n.p[2] = (z == g.Lz - 1) ? s - (long)(g.Lz - 1) * sz : s + sz;
    n.m[2] = (z == 0) ? s + (long)(g.Lz - 1) * sz : s - sz;
    n.p[3] = (t == g.Lt - 1) ? s - (long)(g.Lt - 1) * stt : s + stt;
    n.m[3] = (t == 0) ? s + (long)(g.Lt - 1) * stt : s - stt;
    return n;
}

// Deterministic block sum of two doubles into partials[2*slot + {0,1}].
template <int NT>
__device__ __forceinline__ void block_sum2(double a, double b, double *partials, int slot) {
    static_assert(NT % 64 == 0, "wave64 blocks");
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
    if (threadIdx.x == 0) {
        double A = 0, B = 0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) {
            A += sa[i];
            B += sb[i];
        }
        partials[2 * slot] = A;
        partials[2 * slot + 1] = B;
    }
}

}  // namespace lgf
