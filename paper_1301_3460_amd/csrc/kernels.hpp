// Launch interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace lgf {

// Solver state kept on the device so that a batch of sweeps can be enqueued
// without reading anything back; every sweep kernel returns at once when
// `done` is set.
struct dev_status {
    double F, theta, theta_prev;
    double theta_min;  // smallest theta of the phase
    int n;          // gauge updates applied in the current phase
    int done;       // 1: stop (kernels become no-ops)
    int code;       // 0 running, 1 converged, 4 max_iter, 5 non-finite, 6 diverging
    int rises;      // consecutive iterations with rising theta
    int hist_base;  // history slot of this phase's n = 0
    int since_min;  // sweeps since theta last reached a new minimum
};

// ST_STALLED: theta stopped reaching new minima (the FP32 phase of a mixed
// solve has hit its rounding floor; the solve hands over to FP64).
enum {
    ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXITER = 4, ST_NONFINITE = 5, ST_DIVERGING = 6,
    ST_STALLED = 7
};
// Divergence: theta rose DIVERGE_RISES sweeps in a row and exceeds
// DIVERGE_GROWTH times its smallest value so far (plain steepest descent lets
// theta rise for a while as F still increases, so rises alone are no test).
constexpr int DIVERGE_RISES = 8;
constexpr double DIVERGE_GROWTH = 100.0;

// Stopping test after a sweep kernel: a one-block kernel sums the per-block
// partials in fixed order and updates the device status (enabled == 0: the
// sweep kernel only writes its partials).
struct fin_params {
    double normF, normT, tol;
    int max_iter, increment, hist_cap, enabled;
    int stall;  // > 0: stop with ST_STALLED after this many sweeps without a new minimum
    double *histF, *histT;
};

// Component arrays of links and Fourier fields are S = V + SOA_PAD elements
// apart: an odd number of 128-byte lines (FP32; twice that in FP64) beyond the
// volume, so the same site's lines in the 28 arrays a sweep kernel streams
// fall into different L2 sets instead of all into one.
constexpr long SOA_PAD = 592;

struct geom {
    int Lx, Ly, Lz, Lt;
    long V;
    long S = 0;  // component stride of the SoA arrays (V + SOA_PAD)
    // site-kernel tiling (see block_site): 0 consecutive sites; 1 64 xy-sites
    // x 4 t (needs Lx*Ly % 64 == 0, Lt % 4 == 0), in groups of sgroup segments
    int tblock = 0, sgroup = 1;
    // slices of 4 t in each XCD's range of blocks, walked inside z when > 1
    int tslab = 1;
    // working link format, reals per link: 12 (rows 0,1; row 2 rebuilt), 18
    // (all three rows) or 8 (the minimal form of su3.hpp)
    int lf = 12;
    // gauge group SU(nc), nc = 3 or 2, and the number of complex Fourier
    // fields carrying Delta (4 for SU(3), 2 for SU(2))
    int nc = 3, nf = 4;
    // 1: FP64 sweeps keep the Fourier field (Delta, L Delta) in FP32
    int ff32 = 0;
};

constexpr int SITE_BLOCK = 256;  // threads per block of the site kernels
inline int site_blocks(long V) { return (int)((V + SITE_BLOCK - 1) / SITE_BLOCK); }

// Geometry of lattice L = {Lx, Ly, Lz, Lt} for SU(nc): 12-real links, FP64
// field.  The site-kernel tiling takes 64 consecutive xy-sites x 4 t per
// block where the shape allows it (8x8 xy tiles keep more neighbours in a
// block, but their short rows cost more in DRAM efficiency than they save).
inline geom make_geom(const int L[4], int nc) {
    geom g{};
    g.Lx = L[0];
    g.Ly = L[1];
    g.Lz = L[2];
    g.Lt = L[3];
    g.V = (long)L[0] * L[1] * L[2] * L[3];
    g.S = g.V + SOA_PAD;
    g.nc = nc;
    g.nf = nc == 3 ? 4 : 2;
    g.lf = 12;
    g.ff32 = 0;
    g.tblock = ((long)L[0] * L[1] % 64 == 0 && L[3] % 4 == 0) ? 1 : 0;
    const long nseg = (long)L[0] * L[1] / 64;
    g.sgroup = (nseg % 4 == 0) ? 4 : (nseg % 2 == 0) ? 2 : 1;
    // the 8 XCD ranges split the slices of 4 t evenly
    const int nslab = L[3] / 4;
    g.tslab = (g.tblock && nslab % 8 == 0 && nslab > 8) ? nslab / 8 : 1;
    return g;
}

// All launchers enqueue on `st` and return hipGetLastError().
template <class T>
hipError_t launch_pack_links(const double *Uaos, void *L, const geom &g, hipStream_t st);
hipError_t launch_unpack_links(const void *L64, double *Uaos, const geom &g, hipStream_t st);

template <class T>
hipError_t launch_div_reduce(const geom &g, const void *L, void *D, double *partials,
                             dev_status *status, const fin_params &fp, hipStream_t st);

// exact: g(x) = exp((alpha/2) L Delta) exactly, precomputed into GX (SU(3):
// 6 complex entries per site, stride S; SU(2) evaluates it in the update).
// T = float (the FP32 sweeps of a mixed solve): G is the accumulated
// transformation.  SU(3): Lin holds the constant FP32 copy U0 of the input
// links and GX the transformation after this sweep's step (g(x) G(x), rows
// 0,1, accumulated beforehand by launch_fft_xy_inv_acc or launch_gauge_acc;
// G is the one before it, only checked); the new links G U0 G^dagger are
// formed in the update and not stored (Lout unused).  SU(2): links go from
// Lin to Lout and G is updated in place.
template <class T>
hipError_t launch_update(const geom &g, const void *Lin, void *Lout, const void *LD, void *Dout,
                         void *G, T c, bool exact, void *GX, double *partials, dev_status *status,
                         const fin_params &fp, hipStream_t st);

// One-axis pass of the 4D transform: a block holds W consecutive elements of
// the axis's inner range (the sites below the axis: none for x, x for y, the
// (x,y) plane for z and t) x the whole axis x B consecutive slices (the sites
// above the axis; for t, the z slices), so every HBM access is a contiguous
// row.  Element (w, j, b) sits at w + j*sj + b*sb from the block's first
// element, and in LDS at b*PB + j*PW + w.
struct axis_plan {
    int N = 0;           // extent of the axis
    int W = 1, B = 1;    // inner elements and slices per block
    int nslice = 1;      // slices in total (a multiple of B)
    int PW = 1, PB = 1;  // LDS strides of an axis position and of a slice
    long R = 1;          // length of the inner range (the last row may be ragged)
    long sj = 0, sb = 0; // HBM strides of the axis and of a slice, in elements
    size_t lds = 0;      // LDS bytes per block
};
// A pass over two axes a and b held together in LDS: per block W consecutive
// inner elements (HBM stride 1) x Na x Nb, one inner group and one outer
// slice; the LDS element (w, ja, jb) is at w + ja*PA + jb*PB.
struct tile2_plan {
    int Na = 0, Nb = 0, W = 1;
    long sa = 0, sb = 0;     // HBM strides of axes a and b, in elements
    long R = 1;              // inner extent (the last group may be ragged)
    int ngrp = 1;            // inner groups (R / W rounded up)
    int nouter = 1;          // outer slices
    long so = 0;             // HBM stride of an outer slice
    int PA = 1, PB = 1;      // LDS strides along a and b
    int ta = 0, tb = 0;      // offsets of the axis tables of a and b (twiddles, p2)
    int tw = 0, to = 0;      // offsets of the p2 tables of the inner and the outer axis
    int rmax = 16;           // register tier of the larger of Na, Nb
    int nthr = 512;          // threads per block (1024 when one block fills a compute unit)
    size_t lds = 0;          // LDS bytes per block
};
// How the 4D transform of a context is split into passes.
struct fft_plan {
    // (x,y): 0 register-column kernel (both extents up to 32), 1 whole plane in
    // LDS, 2 an x pass and a y pass
    int xy = 0;
    size_t lds_xy = 0;  // LDS bytes of the (x,y) kernel (modes 0 and 1)
    // (z,t): register-column kernel (both extents up to 32, W consecutive
    // xy-sites per block), else a z pass and a t pass
    bool rc = false;
    int W = 1;
    size_t lds = 0;
    axis_plan x, y, z, t;
    // FP64 32 x 32 register-column passes with two tiles per block (the
    // scaled (z,t) round trip and both (x,y) directions), where half the
    // tile count still gives every compute unit two blocks
    bool xy2 = false, zt2 = false;
    size_t lds_zt2 = 0;
    // FP64, (z,t) beyond the register columns: (x,t) planes as the first and
    // last pass (t2a) and (y,z) tiles of W x-sites as the middle pass (t2b),
    // three passes over the field instead of the five of the x,y / z / t / z /
    // x,y scheme
    bool t2 = false;
    tile2_plan t2a, t2b;
};
// ncu: compute units of the device (0: no two-tile passes)
template <class T> fft_plan plan_fft(const geom &g, size_t zt_lds_budget, int ncu);
// every kernel of the plan fits the LDS of a compute unit and its grid limits
bool fft_plan_fits(const fft_plan &p);
template <class T> void fft_set_max_lds(const geom &g, const fft_plan &p);
// LDS limit of the FP32 update that shares links through LDS (once per process
// and device is enough; repeating it is harmless)
void update_set_max_lds();
// Twiddle tables: one buffer per real type with the axis tables
// exp(-2 pi i j / L_mu), j < L_mu, of x, y, z and t one after the other.
// (x,y) transform, dir -1 forward, +1 inverse
template <class T>
hipError_t launch_fft_xy(const geom &g, void *D, int dir, const void *tw, const fft_plan &pl,
                         const dev_status *status, hipStream_t st);
// Inverse (x,y) pass fused with G(x) <- g(x) G(x) (FP32 sweeps of an SU(3)
// mixed solve; L Delta itself is not stored), when xy_acc_fusable: register-
// column planes with all 4 fields in one block, or wider planes whose 4
// fields fit in LDS together.
template <class T> bool xy_acc_fusable(const geom &g, const fft_plan &pl);
template <class T>
hipError_t launch_fft_xy_inv_acc(const geom &g, void *D, const void *tw, const fft_plan &pl,
                                 const void *Gold, void *Gnew, double c, bool exact,
                                 const dev_status *status, hipStream_t st);
// G(x) <- g(x) G(x) from the field L Delta as a kernel of its own (FP32 sweeps
// of an SU(3) mixed solve whose inverse (x,y) pass cannot take it)
hipError_t launch_gauge_acc(const geom &g, const void *LD, const void *Gold, void *Gnew, double c,
                            bool exact, const dev_status *status, hipStream_t st);
// (z,t) transform.  mode 0: forward, scale by p2max/(V p2), inverse; -1:
// forward only; +1: inverse only
template <class T>
hipError_t launch_fft_zt(const geom &g, void *D, int mode, const void *tw, const T *ptab,
                         T p2max_over_V, const fft_plan &pl, const dev_status *status,
                         hipStream_t st);

// natural <-> transform-position order of 4 fields with component strides
// si (input) and so (output); to_natural: positions -> natural order
hipError_t launch_reorder_fields(const geom &g, const double2 *in, long si, double2 *out, long so,
                                 int to_natural, hipStream_t st);

// F = normF sum Re Tr U and theta = normT sum Tr[Delta Delta^+] of the
// complex128 AoS links Uaos ([4][V][3][3], rows 0,1 read) into out[0..1]
// (device), with the block partials in `partials` (site_blocks(V) pairs): the
// arithmetic of launch_div_reduce + launch_reduce_only on packed links, in
// the same order, without packing them (nothing is allocated or written
// besides partials and out).
hipError_t launch_measure_aos(const geom &g, const double *Uaos, double *partials, double *out,
                              double normF, double normT, hipStream_t st);

hipError_t launch_finalize(const double *partials, int nparts, dev_status *status,
                           const fin_params &fp, hipStream_t st);
hipError_t launch_status_reset(dev_status *status, int hist_base, hipStream_t st);
hipError_t launch_reduce_only(const double *partials, int nparts, double *out2, hipStream_t st);

hipError_t launch_g_identity(void *G32, const geom &g, hipStream_t st);
hipError_t launch_switch(const geom &g, const void *G32, const double *U0aos, void *L64,
                         hipStream_t st);
// launch_switch (SU(3)) fused with launch_div_reduce<double> of its links:
// the same links, field, partials and stopping test
hipError_t launch_switch_div(const geom &g, const void *G32, const double *U0aos, void *L64,
                             void *D, double *partials, dev_status *status, const fin_params &fp,
                             hipStream_t st);

hipError_t launch_field_from_matrix(const double *Maos, void *D64, long V, long S, hipStream_t st);
hipError_t launch_matrix_from_field(const void *D64, double *Maos, long V, long S, hipStream_t st);

hipError_t launch_plaquette(const geom &g, const void *L64, double *partials, hipStream_t st);
hipError_t launch_functional_g(const geom &g, const void *L64, const double *gaos,
                               double *partials, hipStream_t st);

// differentiation (FP64)
hipError_t launch_expm_sites(const double *omega, double *gaos, long n, hipStream_t st);
hipError_t launch_rotate_links(const geom &g, const void *Lin, const double *gaos, void *Lout,
                               hipStream_t st);
hipError_t launch_left_multiply_links(const void *Lin, const double *eaos, void *Lout, long V,
                                      long S, hipStream_t st);
hipError_t launch_omega_grad(const geom &g, const void *D64, const double *omega, double *dF,
                             double normF, hipStream_t st);
hipError_t launch_theta_grad(const geom &g, const void *L64, const void *D64, const double *eps,
                             double *dth, double normT, hipStream_t st);

// SU(2) kernels (su2.hip); the generic launchers above dispatch to them when
// g.nc == 2.
template <class T>
hipError_t launch_pack_su2(const double *Uaos, void *L, const geom &g, hipStream_t st);
hipError_t launch_unpack_su2(const void *L64, double *Uaos, const geom &g, hipStream_t st);
template <class T, class TF>
hipError_t launch_div_reduce_su2(const geom &g, const void *L, void *D, double *partials,
                                 dev_status *status, hipStream_t st);
template <class T, class TF>
hipError_t launch_update_su2(const geom &g, const void *Lin, void *Lout, const void *LD,
                             void *Dout, void *G, T c, bool exact, double *partials,
                             dev_status *status, hipStream_t st);
hipError_t launch_g_identity_su2(void *G32, const geom &g, hipStream_t st);
hipError_t launch_switch_su2(const geom &g, const void *G32, const double *U0aos, void *L64,
                             hipStream_t st);

}  // namespace lgf
