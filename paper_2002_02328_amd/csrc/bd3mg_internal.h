// Internal interface between the host side of libbd3mg (bd3mg_api.hip) and
// its gfx950 kernels (bd3mg_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/bd3mg.h"

namespace bd3mg {

// Records the thread-local message returned by bd3mg_last_error and returns st.
bd3mg_status fail(bd3mg_status st, const char *fmt, ...);

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::bd3mg::fail(BD3MG_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                 __FILE__, __LINE__);                                        \
    } while (0)

#define ST_TRY(expr)                                   \
    do {                                               \
        bd3mg_status s_ = (expr);                      \
        if (s_ != BD3MG_OK) return s_;                 \
    } while (0)

// What the warm-start network needs of a problem: its size, precision, data
// on the device and stream.
struct ProblemView {
    int nx, ny, nz, prec;
    bool data_set;
    const void *y;
    hipStream_t stream;
};
bd3mg_status problem_view(bd3mg_problem p, ProblemView *v);

// Output tile of one workgroup: TX columns (one wavefront wide) by TY rows;
// each of the NT threads owns TY / (NT / TX) = 4 outputs of a column.
constexpr int TX = 64;
constexpr int TY = 16;
constexpr int NT = 256;     // threads per workgroup (4 wavefronts)
constexpr int RMAX = 4;     // largest in-slice kernel radius (kernels up to 9 wide)
constexpr int KZMAX = 9;    // largest kernel extent along z

// Partial sums written per (work item, tile) slot, with d1 = -g, d2 = dp.
//  gradient pass: 0 <g,g>  1 <g,dp>  2 <dp,dp>
//                 3 sum w Dd1.Dd1  4 sum w Dd1.Dd2  5 sum w Dd2.Dd2
constexpr int NQG = 6;
//  direction pass: 0 <Hd1,Hd1> 1 <Hd1,Hd2> 2 <Hd2,Hd2>
//                  3 <VZd1,VZd1>  4 <VZd1,VZd2>  5 <VZd2,VZd2>
constexpr int NQD = 6;
//  evaluation: 0 ||g||^2  1 sum sqrt(|Dx|^2 + delta^2)  2 sum (x - clip x)^2  3 ||VZ x||^2
constexpr int NQE = 4;

// One output slice k of a pass, for the block [z0, z0 + n) (block -1 and the
// whole volume for volume passes).
struct Item {
    int k;
    int block;
    int z0;
    int n;
    // update items: the source pairs [h0, h0 + hn) of the launch group's pair
    // list, each (direction slot, block) whose stored H d1, H d2 on slice k
    // enter H d' on slice k; direction units: the first direction item h0 and
    // the hn (1 or 2) consecutive slices the workgroup takes
    int h0, hn;
    // update items: a copy of the first pair (slot ps, block pb), so that a
    // single-source item starts its loads without a dependent read of the
    // pair list
    int ps, pb;
};

// Work items of one block inside the item lists of a launch group.
struct BlockRange {
    int block;
    int g0, gn;  // gradient-pass items [g0, g0 + gn)
    int d0, dn;  // direction-pass items [d0, d0 + dn)
};

// Block step of the ablation study (Sec. 3.2): BD3MG's subspace step with
// the half-quadratic majorant, or Async-GD / Async-CG (the metric L Id), or
// Async-MM (d' = -A_S(x)^{-1} grad_S f by an inner linear solve).
enum Method : int { M_BD3MG = 0, M_GD = 1, M_CG = 2, M_MM = 3 };

struct Params {
    double lambda, delta, eta, kappa, xmin, xmax;
    double mu;   // curvature inflation of every block majorant (A_S + mu Id)
    int method;  // Method
    double lip;  // L of the metric L Id (M_GD, M_CG)
    int tv3d;    // total variation over (VX, VY, VZ) instead of (VX, VY) per slice
};

struct Geom {
    int nx, ny, nz;
    int rx, ry, rz;
    int R;         // in-slice radius of the device tables: max(rx, ry, 1)
    int ntx, nty;  // tiles per slice of the gradient pass (TX x TY)
    // tile heights (16 or 32 rows) of the direction pass, the update pass and
    // the whole-volume H / adjoint-blur passes
    int ty_dirs, ty_update, ty_aux;
};

// Tiles per slice of a pass with tile height ty.
inline int tiles_of(const Geom &g, int ty) { return g.ntx * ((g.ny + ty - 1) / ty); }

// Device state of a problem, in storage type T.  q holds, slice by slice,
// q_m = XY^T_m (H x - y)_m: the residual blurred in-slice by the adjoint of
// slice m's own factors, so that (H^T (H x - y))_k = sum_c gz_{k+c}[c] q_{k+c}.
template <typename T>
struct DevState {
    T *x, *y, *q, *g, *dp[2];  // dp[0]: previous steps read, dp[1]: written
    const int *stop;           // when non-null and set, every pass returns without writing
    const T *gx, *gy;          // in-slice PSF tables [nz][2R + 1], centred, zero-padded
    const T *gz;               // z PSF table [nz][kz]
    const int *sblk;           // block of every slice
    T *hd[2];                  // H d1, H d2 of the launch group's direction items [slot][ny][nx]
    T *hdw;                    // when set: H d' of each update pair written here by slot (H dp of the next visit)
    int nt;                    // 1: the sweep passes store their volume outputs with the non-temporal hint
};

enum GradMode : int {
    GM_BLOCK = 0,  // g on the items' slices -> s.g, partials NQG
    GM_EVAL = 1,   // no write; partials NQE of ||grad f|| and the non-data terms of f
    GM_ZCOMB = 2,  // out = sum_c gz_{k+c}[c] q_{k+c}  (H^T of the blurred input)
    GM_GRAD = 3    // out = grad f
};

// nshare > 0 (one-tap z table only): q holds nshare shares of the data term
// per item, [share][item][ny][nx], added in order.
template <typename T>
hipError_t launch_grad(const Geom &g, const Params &prm, const DevState<T> &s, const T *q,
                       const T *x, T *out, const Item *items, int nitems, int mode,
                       double *partials, hipStream_t st, int nshare = 0);

// Direction pass over nunits units (slice k of a block with the block's z0,
// n; first direction item h0 and hn = 1 or 2 consecutive slices); stores
// H d1, H d2 of item i at slot i of s.hd (one: only H d1; H d2 = H dp is read
// from slot i of s.hd[1], where the update pass of the previous visit stored it).
template <typename T>
hipError_t launch_dirs(const Geom &g, const Params &prm, const DevState<T> &s, const Item *units,
                       int nunits, double *partials, hipStream_t st, bool one = false);

// Update pass from the stored H d1, H d2 (pairs: (slot, block) per source;
// multi: items may have more than one source, as in a round).
// assign: s.q receives XY^T (H d') on the items' slices (no add, x and dp
// untouched).
template <typename T>
hipError_t launch_update(const Geom &g, const DevState<T> &s, const Item *items, int nitems,
                         const int2 *pairs, const double *u, bool multi, hipStream_t st, int assign = 0);

// Async-MM (Sec. 3.2): the block majorant applied to a block vector p,
//   ap_S = [H^T H p + 2 eta p + lambda V^T Diag(omega(x)) V p + 2 kappa VZ^T VZ p]_S + mu p_S,
// p zero outside each item's block, the data part from qt = XY^T (H p)
// (slices S +- r_z); partials: <p, A p> per (item, tile) slot.  Items are
// the gradient items of a launch group (h0, hn: the block's first item and
// item count in the group).
template <typename T>
hipError_t launch_majapply(const Geom &g, const Params &prm, const DevState<T> &s, const T *qt,
                           const T *x, const T *pv, T *ap, const Item *items, int nitems,
                           double *partials, hipStream_t st);

// Async-MM's inner solve on every block of a launch group: conjugate
// gradients on A_S(x) v = -g_S from v = 0 (for the symmetric A_S the linear
// biconjugate gradient iterates with the shadow residual started at the
// residual are these, bitwise).  Per-block scalars in cgs[CG_STRIDE * block].
enum : int { CG_INIT = 0, CG_VEC = 1, CG_DIR = 2, CG_FINAL = 3 };
constexpr int CG_STRIDE = 10;  // rho[2], done[2], r0, iterations, ||r||^2 at the end, ||g||^2
template <typename T>
struct CgBufs {
    T *r, *p, *v, *ap, *qt;  // residual, direction, solution, A p, XY^T (H p)
    double *pg;              // gradient-pass partials (NQG per slot): <g, g>
    double *pa, *prr;        // <p, A p> and <r, r> per slot
    double *cgs;             // per-block scalars
    double *info;            // per-block info of the step (CG_FINAL)
};
template <typename T>
hipError_t launch_cg(int stage, const Geom &g, const DevState<T> &s, const Item *items, int nitems,
                     const CgBufs<T> &b, int parity, double tol_inner, hipStream_t st);

// qout = XY^T (H src - y) on the items' slices.
template <typename T>
hipError_t launch_refresh(const Geom &g, const DevState<T> &s, const T *src, T *qout,
                          const Item *items, int nitems, hipStream_t st);

// out = H(in) - sub (sub may be null) on the items' slices; with partials,
// each slot also receives its sum of out^2.
template <typename T>
hipError_t launch_H(const Geom &g, const DevState<T> &s, const T *in, const T *sub, T *out,
                    const Item *items, int nitems, double *partials, hipStream_t st);

// out_m = XY^T_m in_m on the items' slices.
template <typename T>
hipError_t launch_blurT(const Geom &g, const DevState<T> &s, const T *in, T *out,
                        const Item *items, int nitems, hipStream_t st);

// General per-depth kernels (dense PSF), pk = [nz][kz][2R+1][2R+1]:
// DM_H    out = H in (- sub, may be null), partials (optional): per (item,
//         tile) sum of out^2;
// DM_DIRS H d1, H d2 of the items' blocks (d1 = -g, d2 = dp) -> s.hd at the
//         item's slot, partials NQD per (item, tile);
// DM_HT   out = H^T in.
// Tiles are TX x g.ty_dirs (16 or 32 rows).
constexpr int RDMAX = 5;    // largest in-slice radius of a dense kernel (11 wide)
constexpr int KZDMAX = 21;  // largest z extent of a dense kernel
enum : int { DM_H = 0, DM_DIRS = 1, DM_HT = 2 };
// nsplit > 1 (DM_HT only, out null): the source slices of every item are
// shared out over nsplit workgroups writing to part ([nsplit][nitems]
// slices), for a reader that adds the shares in order (more workgroups when
// there are few items).
template <typename T>
hipError_t launch_dense(const Geom &g, const Params &prm, const DevState<T> &s, const T *pk,
                        const T *in, const T *sub, T *out, const Item *items, int nitems, int mode,
                        double *partials, hipStream_t st, int nsplit = 1, T *part = nullptr);

// Update pass of the dense mode (the maintained vector is r = Hx - y).
template <typename T>
hipError_t launch_dense_update(const Geom &g, const DevState<T> &s, const Item *items, int nitems,
                               const int2 *pairs, const double *u, hipStream_t st);

// Per block range: fixed-order reduction of the block's slots, the 2x2
// majorant system, its pseudo-inverse and the step coefficients u.
hipError_t launch_solve(const Params &prm, const BlockRange *br, int nbr, int ntiles_g,
                        int ntiles_d, const double *pg, const double *pd, double *u, double *info,
                        const int *stop, hipStream_t st);

// Device stop test after an evaluation pass (see k_check).
hipError_t launch_check(const double *partials, int nslot, double thr, int sweep, int *stop,
                        int *stop_sweep, double *gnorm, hipStream_t st);

// Fixed-order sum of nslot slots of nq doubles into out[nq].
hipError_t launch_sum(const double *partials, int nslot, int nq, double *out, hipStream_t st);

// Bytes of the per-device scratch array of bd3mg_run_noalloc, and its device
// address on a device (taken once per device with hipGetSymbolAddress, that
// device current; later calls return the cached address).
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
hipError_t scratch_base(int device, void **ptr);

// One problem's part of a fused batch pass: every problem's gradient,
// direction, solve or update pass of the same colour index runs in one
// launch, its workgroups from wg0 on (a multiple of 8, so a workgroup's XCD
// is the same as in a launch of its own); owner[h / 8] is the problem of
// workgroup h.  All problems of a fused launch share the precision, the z
// extent, the in-slice radius and the tile heights (template parameters).
template <typename T>
struct FusedArgs {
    Geom g;
    Params prm;
    DevState<T> s;
    const Item *items;      // gradient items, direction units or update items of the colour
    const BlockRange *brs;  // solve: the colour's block ranges
    const int2 *pairs;      // update: source pairs
    double *u;              // solve: written; update: read
    double *pg, *pd;        // gradient and direction partial sums
    double *info;           // solve: per-block info
    int nitems;             // work items (solve: block ranges) of this problem in the pass
    int ntg, ntd;           // solve: tiles per item of the gradient and direction passes
    unsigned wg0;           // first workgroup of this problem in the fused grid
    unsigned gx, gy;        // tiles per slice of the pass
};
enum : int { FP_GRAD = 0, FP_DIRS = 1, FP_SOLVE = 2, FP_UPDATE = 3 };
template <typename T>
hipError_t launch_fused(int pass, const Geom &g, const FusedArgs<T> *fa, const unsigned char *owner, unsigned nwg,
                        hipStream_t st, bool one = false);

// Start and stop events for the next kernel launch of this host thread (set
// around a profiled single-kernel pass, null otherwise): the launchers then
// use hipExtLaunchKernelGGL, which timestamps the kernel's own start and end
// rather than adding event packets to the stream.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

// Streaming copy of n 16-byte words (bandwidth probe), in one of
// COPY_VARIANTS launch shapes (words per lane in flight, workgroups).
constexpr int COPY_VARIANTS = 4;
hipError_t launch_copy(const void *src, void *dst, size_t n16, int variant, hipStream_t st);

}  // namespace bd3mg
