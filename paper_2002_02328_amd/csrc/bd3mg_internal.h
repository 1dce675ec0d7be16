// Internal interface between the host side of libbd3mg (bd3mg_api.hip) and
// its gfx950 kernels (bd3mg_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace bd3mg {

// Output tile of one workgroup: TX columns (one wavefront wide) by TY rows.
constexpr int TX = 64;
constexpr int TY = 16;
constexpr int NT = 256;     // threads per workgroup (4 wavefronts)
constexpr int RMAX = 4;     // largest in-slice kernel radius (kernels up to 9 wide)
constexpr int KZMAX = 9;    // largest kernel extent along z

// Number of double partial sums each workgroup slot writes for a block.
//  0 <g,g>        1 <g,dp>        2 <dp,dp>            (gradient pass)
//  3 <Hd1,Hd1>    4 <Hd1,Hd2>     5 <Hd2,Hd2>          (direction pass)
//  6 sum w Dd1.Dd1  7 sum w Dd1.Dd2  8 sum w Dd2.Dd2
//  9 <VZd1,VZd1>  10 <VZd1,VZd2>  11 <VZd2,VZd2>
constexpr int NQ = 12;
// Partial sums of the evaluation pass:
//  0 ||g||^2  1 ||r||^2  2 sum sqrt(|Dx|^2 + delta^2)  3 sum (x - clip x)^2  4 ||VZ x||^2
constexpr int NE = 5;

// A run of consecutive z-slices handled by one column of workgroups: a block
// of the partition, or a chunk of the volume for whole-volume passes.
struct Segment {
    int z0;
    int n;
    int block;   // block index (or -1 for volume chunks)
    int parity;  // which previous-step buffer holds the block's last step
};

struct Params {
    double lambda, delta, eta, kappa, xmin, xmax;
};

struct Geom {
    int nx, ny, nz;
    int rx, ry, rz;
    int ntx, nty;  // tiles per slice
};

// Device state of a problem, in storage type T.
template <typename T>
struct DevState {
    T *x, *y, *r, *g, *dp[2];
    const T *gx, *gy, *gz;  // PSF tables [nz][k]
};

enum GradMode : int {
    GM_BLOCK = 0,  // write g on the block, partial sums 0..2
    GM_EVAL = 1,   // no write; evaluation partial sums of f and ||grad f||
    GM_HT = 2,     // write H^T r into out
    GM_GRAD = 3    // write grad f into out
};

template <typename T>
hipError_t launch_grad(const Geom &g, const Params &prm, const DevState<T> &s, const T *rin,
                       T *out, const Segment *segs, int nseg, int mode, double *partials,
                       hipStream_t st);

template <typename T>
hipError_t launch_dirs(const Geom &g, const Params &prm, const DevState<T> &s,
                       const Segment *segs, int nseg, double *partials, hipStream_t st);

template <typename T>
hipError_t launch_update(const Geom &g, const DevState<T> &s, const Segment *segs, int nseg,
                         const double *u, hipStream_t st);

// out = H(in) - sub (sub may be null) on the slices of the segments.
template <typename T>
hipError_t launch_H(const Geom &g, const DevState<T> &s, const T *in, const T *sub, T *out,
                    const Segment *segs, int nseg, hipStream_t st);

// Per block: fixed-order sum of its workgroup partials, the 2x2 majorant
// system, its pseudo-inverse and the step coefficients u (2 doubles per block).
hipError_t launch_solve(const Params &prm, const Segment *segs, int nseg, int slots_per_seg,
                        const double *partials, double *u, double *info, hipStream_t st);

// Fixed-order sum of nslot evaluation slots of NE doubles into out[NE].
hipError_t launch_sum_eval(const double *partials, int nslot, double *out, hipStream_t st);

// Streaming copy of n 16-byte words (bandwidth probe).
hipError_t launch_copy(const void *src, void *dst, size_t n16, hipStream_t st);

}  // namespace bd3mg
