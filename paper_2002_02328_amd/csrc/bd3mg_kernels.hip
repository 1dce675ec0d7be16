// gfx950 kernels of libbd3mg: the per-block work of one BD3MG update
// (Sec. 2.3, box "Worker", for the criterion of Sec. 3.1).
//
// Layout and decomposition.  Volumes are [nz][ny][nx], x fastest.  Every pass
// is split into independent work items, one output slice each, and a
// workgroup computes one TX x TY tile of one item: a launch has (tiles per
// slice) x (items) workgroups, enough to fill the 256 CUs even for a single
// colour of blocks.  Global rows are read 64 consecutive elements at a time
// (one wavefront, coalesced); in-slice halos go through LDS, where the
// separable depth-variant blur runs as an x pass then a y pass.
//
// The z extent KZ and the in-slice radius R of the PSF are template
// parameters: every tile loop has a compile-time trip count, so each thread
// issues all global loads of a stencil before it waits for any of them, and
// the filter taps sit in registers.  In-slice tables are stored with 2R + 1
// taps per slice (zero-padded when kx != ky).
//
// The residual enters only through q_m = XY^T_m (H x - y)_m (each slice
// blurred by the adjoint of its own in-slice factors), so the data part of
// the gradient is a pure z-stencil, (H^T r)_k = sum_c gz_{k+c}[c] q_{k+c},
// and the update pass keeps q current: q_m += XY^T_m (H d')_m.
//
// Inner products are accumulated in double: per thread in index order, a
// fixed DPP sum per wavefront, the four wavefronts in order, then the slots of a
// block in slot order (k_solve) -- a fixed order, so runs are bitwise
// reproducible.
#include <hip/hip_ext.h>
#include <mutex>

#include "bd3mg_internal.h"

namespace bd3mg {

namespace {

constexpr int RPT = TY / (NT / TX);  // outputs (rows) per thread of a TY-row tile: 4

__device__ __forceinline__ size_t vidx(const Geom &g, int k, int j, int i)
{
    return ((size_t)k * g.ny + j) * g.nx + i;
}

template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi) { return v < lo ? lo : (v > hi ? hi : v); }

// 1 / sqrt(v): the hardware reciprocal square root in single precision
// (about 1 ulp), the correctly rounded quotient in double precision.  The
// single-precision instruction flushes subnormal arguments, so v is held at
// or above the smallest normal number (every argument here is at least
// delta^2, a normal number for any delta above 1.1e-19); above it this is
// the instruction rsqrtf takes there, with none of its rescaling.
__device__ __forceinline__ float inv_sqrt(float v) { return __builtin_amdgcn_rsqf(fmaxf(v, 0x1p-126f)); }
__device__ __forceinline__ double inv_sqrt(double v) { return 1.0 / sqrt(v); }

// Tile row of a thread's e-th output when each thread owns NR consecutive
// rows of one column (wavefront w holds rows [w NR, (w + 1) NR)).
template <int NR>
__device__ __forceinline__ int out_row(int e) { return (int)(threadIdx.x / TX) * NR + e; }

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// Element e = threadIdx.x + q NT of a W x H region whose corner is at global
// (y0 - HY, x0 - HX): the in-slice offset j nx + i of the element, or 0 (a
// valid address) when it lies outside the slice or past the region, with a
// flag.  Loads through off[] need no branch: the value is kept or zeroed by a
// select.  Element e sits at index e of a W-wide LDS tile padded to E NT.
template <int W, int H, int HX, int HY>
struct Region {
    static constexpr int N = W * H;
    static constexpr int E = cdiv(N, NT);
    static constexpr int PAD = E * NT;  // LDS elements to allocate
    uint32_t off[E];  // element offset in the slice (non-negative, < 2^30)
    bool inb[E];
    __device__ __forceinline__ Region(const Geom &g, int x0, int y0)
    {
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int e = threadIdx.x + q * NT;
            const int jj = e / W, ii = e - jj * W;
            const int j = y0 - HY + jj, i = x0 - HX + ii;
            inb[q] = e < N && i >= 0 && i < g.nx && j >= 0 && j < g.ny;
            off[q] = inb[q] ? (uint32_t)(j * g.nx + i) : 0u;
        }
    }
};

template <int W, int H>
constexpr int padded() { return cdiv(W * H, NT) * NT; }

// base[eoff] with the byte offset formed in 32 bits: base is uniform across
// the workgroup, so the load takes the scalar-base plus 32-bit vector-offset
// form and needs no 64-bit address arithmetic per element.
template <typename T>
__device__ __forceinline__ T ldo(const T *base, uint32_t eoff)
{
    return *(const T *)((const char *)base + eoff * (uint32_t)sizeof(T));
}

// Buffer descriptor of n elements from p (gfx9 format word): loads through it
// take the base in scalar registers and a 32-bit byte offset in a vector
// register, so the many loads of a slice that share per-thread offsets need
// no 64-bit address arithmetic each (the plain pointer form above loses the
// scalar base once the offsets are hoisted out of a loop).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_of(const T *p, size_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)(n * sizeof(T)), 0x00020000);
}

template <typename T>
__device__ __forceinline__ T ldbuf(__amdgpu_buffer_rsrc_t r, uint32_t boff);
template <>
__device__ __forceinline__ float ldbuf<float>(__amdgpu_buffer_rsrc_t r, uint32_t boff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0));
}
template <>
__device__ __forceinline__ double ldbuf<double>(__amdgpu_buffer_rsrc_t r, uint32_t boff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}

// Stores of the passes' volume outputs; STREAM: with the non-temporal hint
// (cache policy bit nt), which streams them through the caches instead of
// keeping them there. It pays when the volumes a colour touches are far
// larger than the caches and costs when the next pass would find them there.
template <bool STREAM = false>
__device__ __forceinline__ void stbuf(__amdgpu_buffer_rsrc_t r, uint32_t boff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, boff, 0, STREAM ? 2 : 0);
}
template <bool STREAM = false>
__device__ __forceinline__ void stbuf(__amdgpu_buffer_rsrc_t r, uint32_t boff, double v)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, boff, 0, STREAM ? 2 : 0);
}

// x pass from I (rows of width WI, at least ROWS rows) to O (rows of width WO,
// padded to a multiple of NT), WO output columns over ROWS rows:
//   forward O[r][c] = sum_a wx[a] I[r][c + OFF - a],
//   adjoint O[r][c] = sum_a wx[a] I[r][c + OFF + a].
// Elements past the last row recompute the last row into the padding.
template <typename T, int R, int WI, int WO, int ROWS, int OFF, bool ADJ>
__device__ __forceinline__ void xpass(const T *I, T *O, const T (&wx)[2 * R + 1])
{
    constexpr int N = WO * ROWS, E = cdiv(N, NT);
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int e = threadIdx.x + q * NT;
        int r = e / WO;
        const int c = e - r * WO;
        if (q == E - 1) r = r < ROWS ? r : ROWS - 1;
        const T *row = I + r * WI + c + OFF;
        T acc = 0;
#pragma unroll
        for (int a = -R; a <= R; ++a) acc += wx[a + R] * row[ADJ ? a : -a];
        O[e] = acc;
    }
}

// Row stride of an LDS tile W elements wide whose rows are read 16 bytes at
// a time: W rounded up to a whole number of 16-byte words.
template <typename T, int W>
constexpr int vstride() { return cdiv(W * (int)sizeof(T), 16) * 16 / (int)sizeof(T); }

// LDS index of region element e (row e / W, column e % W) in a tile of row
// stride WS.
template <int W, int WS>
__device__ __forceinline__ int lds_at(int e)
{
    const int r = e / W;
    return r * WS + (e - r * W);
}

// x pass to TX output columns, four consecutive outputs per thread: from I
// (rows of stride WS = vstride<T, TX + 2R>(), 16-byte aligned; column c of
// the output tile reads columns c .. c + 2R) to O (rows of width TX), over
// ROWS rows:
//   forward O[r][c] = sum_a wx[a] I[r][c + R - a],
//   adjoint O[r][c] = sum_a wx[a] I[r][c + R + a].
// The 4 + 2R inputs of a thread are read as whole 16-byte words.
template <typename T, int R, int ROWS, bool ADJ>
__device__ __forceinline__ void xpass4(const T *I, T *O, const T (&wx)[2 * R + 1])
{
    constexpr int WS = vstride<T, TX + 2 * R>();
    constexpr int VW = 16 / (int)sizeof(T);  // elements per 16-byte word
    constexpr int NI = 4 + 2 * R, NL = cdiv(NI, VW);
    static_assert(TX % 4 == 0 && WS % VW == 0 && (TX - 4) + NL * VW <= WS, "x pass reads stay in the row");
    constexpr int G = TX / 4, N = G * ROWS, E = cdiv(N, NT);
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int e = threadIdx.x + q * NT;
        if (N % NT != 0 && e >= N) break;
        const int r = e / G, c = 4 * (e - r * G);
        T in[NL * VW];
        const uint4 *src = reinterpret_cast<const uint4 *>(I + r * WS + c);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const uint4 w = src[l];
            __builtin_memcpy(in + l * VW, &w, 16);
        }
        T out[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            T acc = 0;
#pragma unroll
            for (int a = -R; a <= R; ++a) acc += wx[a + R] * in[v + R + (ADJ ? a : -a)];
            out[v] = acc;
        }
        uint4 *dst = reinterpret_cast<uint4 *>(O + r * TX + c);
#pragma unroll
        for (int l = 0; l < 4 / VW; ++l) {
            uint4 w;
            __builtin_memcpy(&w, out + l * VW, 16);
            dst[l] = w;
        }
    }
}

// y pass into registers: v[e] at tile row out_row<NR>(e), column
// threadIdx.x % TX, reading rows (out_row + OFF -/+ b) of B (rows of width
// WB).  A thread's NR rows are consecutive, so it reads the NR + 2R values of
// its column once and slides the stencil over them.
template <typename T, int R, int WB, int OFF, bool ADJ, int NR>
__device__ __forceinline__ void ypass_out(const T *B, T (&v)[NR], const T (&wy)[2 * R + 1])
{
    const int i = threadIdx.x & (TX - 1);
    const T *col = B + (out_row<NR>(0) + OFF - R) * WB + i;
    T c[NR + 2 * R];
#pragma unroll
    for (int t = 0; t < NR + 2 * R; ++t) c[t] = col[t * WB];
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        T acc = 0;
#pragma unroll
        for (int b = -R; b <= R; ++b) acc += wy[b + R] * c[e + R + (ADJ ? b : -b)];
        v[e] = acc;
    }
}

template <typename T, int R>
__device__ __forceinline__ void load_taps(T (&w)[2 * R + 1], const T *__restrict__ t)
{
#pragma unroll
    for (int a = 0; a < 2 * R + 1; ++a) w[a] = t[a];
}

// One DPP move of a double (both halves with the same lane pattern). Lanes of
// rows outside ROWS are not written and hold whatever the destination held
// (no zeroing move per half): callers use no value that passes through them.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront in registers: butterflies inside each
// row of 16 lanes (quad permutes, half-row and row mirrors: every lane ends
// with its row's sum), then the two row broadcasts. Only lane 63's result is
// the total, and only it may be used: the broadcast steps add undefined values
// in the rows they do not write (rows 0 and 2, then 0 and 1), and lane 63
// reads only lane 47 (row 2 before its undefined add) and lane 31 (row 1,
// written by the first broadcast).
__device__ __forceinline__ double wave_sum_last(double s)
{
    s += dpp_move<0xb1, 0xf>(s);   // quad_perm [1,0,3,2]
    s += dpp_move<0x4e, 0xf>(s);   // quad_perm [2,3,0,1]
    s += dpp_move<0x141, 0xf>(s);  // row_half_mirror
    s += dpp_move<0x140, 0xf>(s);  // row_mirror
    s += dpp_move<0x142, 0xa>(s);  // row_bcast:15 into rows 1 and 3
    s += dpp_move<0x143, 0xc>(s);  // row_bcast:31 into rows 2 and 3
    return s;
}

// Workgroup reduction of NV doubles (DPP sum per wavefront, then the
// wavefronts in order); thread v < NV stores the total of value v to dst[v].
// Values v >= nlive are zero on every thread (a uniform condition) and are
// stored as 0 without their wavefront sums.
template <int NV>
__device__ __forceinline__ void wg_reduce_store(double (&q)[NV], double *red, double *dst, int nlive = NV)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = 0.0;
        if (v < nlive) s = wave_sum_last(q[v]);
        if (lane == 63) red[wave * NV + v] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w * NV + threadIdx.x];
        dst[threadIdx.x] = s;
    }
}

// Block index and grid of a workgroup as a pass sees them: the hardware's
// own for a pass launched alone, or the part of a fused launch (several
// problems' passes in one grid) that belongs to one problem.
struct VB {
    unsigned x, y, z, gx, gy, gz;
};

__device__ __forceinline__ VB vb_native()
{
    return VB{blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gridDim.y, gridDim.z};
}

// Tile (x, y) and item (z) of this workgroup, XCD-aware: the dispatcher
// hands linear workgroup h to XCD h mod 8, so each XCD's workgroups are
// mapped here to one contiguous run of the (x, y, z) order (a bijection of
// the grid). Neighbouring tiles of a slice then run on the same XCD, and the
// halo rows they share are found in that XCD's L2 (the update pass, whose
// reads are one source slice per item with its halo).  (A fused launch
// starts each problem's part at a multiple of 8, so h mod 8 is still the
// XCD.)
__device__ __forceinline__ uint3 xcd_block(const VB &v)
{
    constexpr unsigned NXCD = 8;
    const unsigned gx = v.gx, gxy = v.gx * v.gy, n = gxy * v.gz;
    const unsigned h = v.x + gx * v.y + gxy * v.z;
    const unsigned per = n / NXCD, rem = n % NXCD, c = h % NXCD;
    const unsigned t = c * per + min(c, rem) + h / NXCD;
    return make_uint3(t % gx, (t / gx) % v.gy, t / gxy);
}

// Tile of this workgroup within its slice, XCD-aware: when a slice has a
// multiple of 8 tiles, the plain order sends tile l of every slice to XCD
// l mod 8 (no two neighbouring tiles on one XCD); here XCD c takes instead
// the contiguous tiles [c n/8, (c + 1) n/8) of each slice, neighbours that
// share their halos in its L2, still slice after slice, so the same tile of
// consecutive slices (which share source slices) stays on one XCD, n/8
// workgroups apart.
__device__ __forceinline__ uint2 xcd_slice_tile(const VB &v)
{
    const unsigned gx = v.gx, n = v.gx * v.gy;
    unsigned l = v.x + gx * v.y;
    if (n % 8 == 0) l = (l % 8) * (n / 8) + l / 8;
    return make_uint2(l % gx, l / gx);
}

__device__ __forceinline__ size_t slot_of(const VB &v)
{
    return ((size_t)v.z * v.gy + v.y) * v.gx + v.x;
}

}  // namespace

// ---------------------------------------------------------------------------
// Gradient pass, one output slice k per item:
//   (H^T r)_k = sum_c gz_{k+c}[c] q_{k+c}
//   g = H^T r + lambda (VX^T(w VX x) + VY^T(w VY x)) + 2 eta (x - clip x)
//       + 2 kappa VZ^T VZ x,     w = 1 / sqrt((VX x)^2 + (VY x)^2 + delta^2)
// and with the total variation taken along z too (TV3), w = 1 / sqrt((VX x)^2
// + (VY x)^2 + (VZ x)^2 + delta^2) and lambda VZ^T(w VZ x) added, which needs
// x on slices k - 1 and k + 1 as well.
// g is formed on the tile plus one column and one row beyond it, so the
// curvature sums of the block's total-variation majorant, which need the
// forward differences of g and dp, come out of the same workgroup.
// GM_BLOCK writes g to s.g with <g,g>, <g,dp>, <dp,dp> and, with d1 = -g and
// d2 = dp, sum w (VX d_a VX d_b + VY d_a VY d_b); GM_GRAD writes g to out;
// GM_EVAL sums ||g||^2 and the TV, box and z terms of f; GM_ZCOMB writes only
// the z-stencil of q to out.
// ---------------------------------------------------------------------------
// BLK: the sweep's mode GM_BLOCK fixed at compile time (its instance carries
// no code of the other modes and no copies of their sums); otherwise mode_in.
// STREAM: g stored with the non-temporal hint (s.nt).
template <typename T, int KZ, bool TV3, bool BLK, bool STREAM = false>
__device__ __forceinline__ void grad_body(const VB vb, Geom g, Params prm, DevState<T> s, const T *__restrict__ q,
                                          const T *__restrict__ x, T *__restrict__ out,
                                          const Item *__restrict__ items, int mode_in,
                                          double *__restrict__ partials, int nshare)
{
    const int mode = BLK ? (int)GM_BLOCK : mode_in;
    constexpr int RZ = KZ / 2;
    constexpr int XW = TX + 3, XH = TY + 3;  // x at (y0-1+jj, x0-1+ii)
    constexpr int PW = TX + 2, PH = TY + 2;  // w VX x, w VY x, w at (y0-1+jj, x0-1+ii)
    constexpr int GW = TX + 1, GH = TY + 1;  // g, dp at (y0+jj, x0+ii)
    __shared__ T X[padded<XW, XH>()];
    __shared__ T PX[padded<PW, PH>()];
    __shared__ T PY[padded<PW, PH>()];
    __shared__ T WW[padded<PW, PH>()];
    __shared__ double red[(NT / 64) * NQG];
    // g and dp on the tile plus one column and row, for the curvature sums,
    // written over x and w VX x once the gradient is formed (four tiles of
    // LDS instead of six: more workgroups fit a compute unit)
    T *const G = X;
    T *const D = PX;
    static_assert(padded<GW, GH>() <= padded<XW, XH>() && padded<GW, GH>() <= padded<PW, PH>(),
                  "g and dp must fit the tiles they replace");
    // TV3: x on slice k - 1 (same positions as X), and at the positions of w
    // the z part w_{k-1} VZ x_{k-1} - w_k VZ x_k of VZ^T(w VZ x)
    __shared__ T XM[TV3 ? padded<XW, XH>() : 1];
    __shared__ T PT[TV3 ? padded<PW, PH>() : 1];

    // tiles in the XCD-aware order within the slice (neighbours share their
    // halos in L2; the same tile of consecutive slices stays on one XCD)
    const uint2 tl = xcd_slice_tile(vb);
    const size_t slot = ((size_t)vb.z * vb.gy + tl.y) * vb.gx + tl.x;
    const Item it = items[vb.z];
    if (s.stop && *s.stop) return;  // read with the item, not before it
    const int k = it.k;
    const int x0 = tl.x * TX, y0 = tl.y * TY;
    const size_t S = (size_t)g.nx * g.ny;
    const bool block = (mode == GM_BLOCK);

    // loads first: x with its halo, q on the KZ slices, dp
    Region<XW, XH, 1, 1> rx(g, x0, y0);
    Region<GW, GH, 0, 0> rg(g, x0, y0);
    T xr[rx.E], ht[rg.E], dv[rg.E];
    if (mode != GM_ZCOMB) {
        const __amdgpu_buffer_rsrc_t xs = buf_of(x + (size_t)k * S, S);
#pragma unroll
        for (int qq = 0; qq < rx.E; ++qq) {
            const T v = ldbuf<T>(xs, rx.off[qq] * (uint32_t)sizeof(T));
            xr[qq] = rx.inb[qq] ? v : T(0);
        }
    }
    constexpr int PE = cdiv(PW * PH, NT);
    T xm[TV3 ? rx.E : 1], xn[TV3 ? PE : 1];
    if constexpr (TV3) {
        if (mode != GM_ZCOMB) {
            // x on slice k - 1 (zero at k = 0) and on slice k + 1 at the
            // positions of w (zero at k = nz - 1)
            const __amdgpu_buffer_rsrc_t xa = buf_of(x + (size_t)max(k - 1, 0) * S, S);
#pragma unroll
            for (int qq = 0; qq < rx.E; ++qq) {
                const T v = ldbuf<T>(xa, rx.off[qq] * (uint32_t)sizeof(T));
                xm[qq] = (rx.inb[qq] && k >= 1) ? v : T(0);
            }
            const Region<PW, PH, 1, 1> rp(g, x0, y0);
            const __amdgpu_buffer_rsrc_t xb = buf_of(x + (size_t)min(k + 1, g.nz - 1) * S, S);
#pragma unroll
            for (int qq = 0; qq < PE; ++qq) {
                const T v = ldbuf<T>(xb, rp.off[qq] * (uint32_t)sizeof(T));
                xn[qq] = (rp.inb[qq] && k < g.nz - 1) ? v : T(0);
            }
        }
    }
    uint32_t bo[rg.E];
#pragma unroll
    for (int qq = 0; qq < rg.E; ++qq) {
        ht[qq] = dv[qq] = 0;
        bo[qq] = rg.off[qq] * (uint32_t)sizeof(T);
    }
    if (block) {
        const __amdgpu_buffer_rsrc_t ds = buf_of(s.dp[0] + (size_t)k * S, S);
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const T v = ldbuf<T>(ds, bo[qq]);
            dv[qq] = rg.inb[qq] ? v : T(0);
        }
    }
    if (KZ == 1 && nshare > 0) {
        // the data term is given as nshare shares per item (the general-kernel
        // adjoint split over workgroups), q = [share][item][ny][nx]: added in order
        for (int p = 0; p < nshare; ++p) {
            const __amdgpu_buffer_rsrc_t qp = buf_of(q + ((size_t)p * vb.gz + vb.z) * S, S);
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) ht[qq] += ldbuf<T>(qp, bo[qq]);
        }
    } else if (sizeof(T) == 4 && (KZ <= 7 || BLK)) {
        // taps past the volume read the nearest slice with weight 0: no
        // branch per tap, so every tap's loads can be in flight together
        // (single precision; the 9-tap block instance takes 86 VGPRs against
        // 56 with a branch per tap and still runs 8 % faster on 512x512x128;
        // the 9-tap instance of the other modes would spill)
#pragma unroll
        for (int c = -RZ; c <= RZ; ++c) {
            const int m = min(max(k + c, 0), g.nz - 1);
            const T w = (k + c == m) ? s.gz[(size_t)m * KZ + (c + RZ)] : T(0);
            const __amdgpu_buffer_rsrc_t qm = buf_of(q + (size_t)m * S, S);
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) ht[qq] += w * ldbuf<T>(qm, bo[qq]);
        }
    } else {
#pragma unroll
        for (int c = -RZ; c <= RZ; ++c) {
            const int m = k + c;
            if (m < 0 || m >= g.nz) continue;
            const T w = s.gz[(size_t)m * KZ + (c + RZ)];
            const __amdgpu_buffer_rsrc_t qm = buf_of(q + (size_t)m * S, S);
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) ht[qq] += w * ldbuf<T>(qm, bo[qq]);
        }
    }
    if (mode == GM_ZCOMB) {
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const int e = threadIdx.x + qq * NT;
            const int lj = e / GW, li = e - lj * GW;
            if (rg.inb[qq] && lj < TY && li < TX) out[(size_t)k * S + rg.off[qq]] = ht[qq];
        }
        return;
    }
#pragma unroll
    for (int qq = 0; qq < rx.E; ++qq) X[threadIdx.x + qq * NT] = xr[qq];
    if constexpr (TV3) {
#pragma unroll
        for (int qq = 0; qq < rx.E; ++qq) XM[threadIdx.x + qq * NT] = xm[qq];
    }
    __syncthreads();
    // w, w VX x and w VY x once per position; zero outside the slice
    const T del2 = (T)(prm.delta * prm.delta);
    {
        constexpr int N = PW * PH, E = cdiv(N, NT);
#pragma unroll
        for (int qq = 0; qq < E; ++qq) {
            const int e = threadIdx.x + qq * NT;
            if (e < N) {
                const int jj = e / PW, ii = e - jj * PW;
                const int j = y0 - 1 + jj, i = x0 - 1 + ii;
                // computed everywhere without a branch: the reads stay inside
                // the x tiles (jj + 1 < XH, ii + 1 < XW), whose elements
                // outside the slice are zero, and the results there are
                // replaced by zero
                const bool in = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
                const T *xc = X + jj * XW + ii;
                const T xv = xc[0];
                const T dxv = (i < g.nx - 1) ? xc[1] - xv : T(0);
                const T dyv = (j < g.ny - 1) ? xc[XW] - xv : T(0);
                T w, pt = 0;
                if constexpr (TV3) {
                    const T dzv = (k < g.nz - 1) ? xn[qq] - xv : T(0);
                    w = inv_sqrt(dxv * dxv + dyv * dyv + dzv * dzv + del2);
                    // w VZ x on slice k - 1 at the same position
                    T zm = 0;
                    if (k >= 1) {
                        const T *mc = XM + jj * XW + ii;
                        const T mv = mc[0];
                        const T dxm = (i < g.nx - 1) ? mc[1] - mv : T(0);
                        const T dym = (j < g.ny - 1) ? mc[XW] - mv : T(0);
                        const T dzm = xv - mv;
                        zm = inv_sqrt(dxm * dxm + dym * dym + dzm * dzm + del2) * dzm;
                    }
                    pt = zm - w * dzv;
                } else {
                    w = inv_sqrt(dxv * dxv + dyv * dyv + del2);
                }
                PX[e] = in ? w * dxv : T(0);
                PY[e] = in ? w * dyv : T(0);
                WW[e] = in ? w : T(0);
                if constexpr (TV3) PT[e] = in ? pt : T(0);
            }
        }
    }
    __syncthreads();

    const T lam = (T)prm.lambda, eta2 = (T)(2.0 * prm.eta), kap2 = (T)(2.0 * prm.kappa),
            lo = (T)prm.xmin, hi = (T)prm.xmax;
    double qs[NQG] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const __amdgpu_buffer_rsrc_t go = buf_of(s.g + (size_t)k * S, S);
    T gr[rg.E];
#pragma unroll
    for (int qq = 0; qq < rg.E; ++qq) {
        const int e = threadIdx.x + qq * NT;
        const int lj = e / GW, li = e - lj * GW;
        // the tile's own outputs inside the slice (the extra row and column
        // are formed for the curvature sums only)
        const bool own = rg.inb[qq] && lj < TY && li < TX;
        T gv = 0;
        if (rg.N % NT == 0 || e < rg.N) {
            // formed without a branch at every element of the region: the
            // reads stay inside the tiles, whose elements outside the slice
            // are zero; g there is replaced by zero, and the sums add exact
            // zeros for all but the tile's own outputs
            const int j = y0 + lj, i = x0 + li;
            const T *xc = X + (lj + 1) * XW + (li + 1);
            const T xv = xc[0];
            // VX^T(w VX x) + VY^T(w VY x) at (j, i); P is zero outside the slice
            const int pc = (lj + 1) * PW + (li + 1);
            T tv = PX[pc - 1] - PX[pc] + PY[pc - PW] - PY[pc];
            if constexpr (TV3) tv += PT[pc];
            const T box = xv - clampv(xv, lo, hi);
            gv = ht[qq] + lam * tv + eta2 * box;
            const size_t o = (size_t)k * S + rg.off[qq];
            T dz = 0;
            if (prm.kappa != 0.0) {
                T zz = 0;
                if (k >= 1) zz += xv - x[o - S];
                if (k < g.nz - 1) {
                    dz = x[o + S] - xv;
                    zz -= dz;
                }
                gv += kap2 * zz;
            } else if (TV3 && mode == GM_EVAL && k < g.nz - 1) {
                dz = x[o + S] - xv;
            }
            gv = rg.inb[qq] ? gv : T(0);
            if (block) {
                const double gd = own ? (double)gv : 0.0, dd = own ? (double)dv[qq] : 0.0;
                qs[0] += gd * gd;
                qs[1] += gd * dd;
                qs[2] += dd * dd;
            } else if (mode == GM_GRAD) {
                if (own) out[o] = gv;
            } else if (own) {  // GM_EVAL: terms of f in double
                const double xd = (double)xv;
                const double dxd = (i < g.nx - 1) ? (double)xc[1] - xd : 0.0;
                const double dyd = (j < g.ny - 1) ? (double)xc[XW] - xd : 0.0;
                const double dzd = (double)dz;
                const double bx = xd - (xd < prm.xmin ? prm.xmin : (xd > prm.xmax ? prm.xmax : xd));
                const double gd = (double)gv;
                qs[0] += gd * gd;
                const double tz = TV3 ? dzd * dzd : 0.0;
                qs[1] += sqrt(dxd * dxd + dyd * dyd + tz + prm.delta * prm.delta);
                qs[2] += bx * bx;
                qs[3] += dzd * dzd;
            }
        }
        gr[qq] = gv;
    }
    if (block) {
        // g of the tile's outputs, stored once the loop is done
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const int e = threadIdx.x + qq * NT;
            const int lj = e / GW, li = e - lj * GW;
            if (rg.inb[qq] && lj < TY && li < TX) stbuf<STREAM>(go, bo[qq], gr[qq]);
        }
        __syncthreads();  // x and w VX x are read no more
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const int e = threadIdx.x + qq * NT;
            if (rg.N % NT != 0 && e >= rg.N) break;
            G[e] = gr[qq];
            D[e] = dv[qq];
        }
        __syncthreads();
        // sum_S w (VX d_a VX d_b + VY d_a VY d_b), d1 = -g, d2 = dp
        const int tx = threadIdx.x & (TX - 1);
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            const int lj = out_row<RPT>(e), li = tx;
            const int j = y0 + lj, i = x0 + li;
            // formed at every row of the tile (the reads stay inside the
            // tiles); outputs outside the slice weigh 0 and add exact zeros
            const double w = (i < g.nx && j < g.ny) ? (double)WW[(lj + 1) * PW + (li + 1)] : 0.0;
            const int c0 = lj * GW + li;
            const double g0 = (double)G[c0], p0 = (double)D[c0];
            const double dx1 = (i < g.nx - 1) ? g0 - (double)G[c0 + 1] : 0.0;
            const double dy1 = (j < g.ny - 1) ? g0 - (double)G[c0 + GW] : 0.0;
            const double dx2 = (i < g.nx - 1) ? (double)D[c0 + 1] - p0 : 0.0;
            const double dy2 = (j < g.ny - 1) ? (double)D[c0 + GW] - p0 : 0.0;
            qs[3] += w * (dx1 * dx1 + dy1 * dy1);
            qs[4] += w * (dx1 * dx2 + dy1 * dy2);
            qs[5] += w * (dx2 * dx2 + dy2 * dy2);
        }
        wg_reduce_store<NQG>(qs, red, partials + slot * NQG);
    } else if (mode == GM_EVAL) {
        double q4[NQE] = {qs[0], qs[1], qs[2], qs[3]};
        wg_reduce_store<NQE>(q4, red, partials + slot * NQE);
    }
}

// Waves per SIMD the register budget aims at: at least four in single
// precision (the block instances' branch-free z taps take 56-86 VGPRs with
// 1-9 taps, five to eight waves; the other modes' instances about 100, and
// a five-wave budget spills them); the LDS holds double precision to three
// (one with 3D TV) and single-precision 3D TV to three.
template <typename T, int KZ, bool TV3, bool BLK, bool STREAM>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? (TV3 ? 1 : 3) : (TV3 ? 3 : 4))))
k_grad(Geom g, Params prm, DevState<T> s, const T *__restrict__ q, const T *__restrict__ x,
       T *__restrict__ out, const Item *__restrict__ items, int mode, double *__restrict__ partials,
       int nshare)
{
    grad_body<T, KZ, TV3, BLK, STREAM>(vb_native(), g, prm, s, q, x, out, items, mode, partials, nshare);
}

// ---------------------------------------------------------------------------
// Per block: fixed-order reduction of its gradient and direction slots, then
// the 2x2 system of the memory-gradient subspace (Sec. 2.3, eq. "minimizer"):
//   B = D^T A_S D with D = [d1 | d2], d1 = -g, d2 = dp,
//   c = D^T g = (-<g,g>, <dp,g>),  u = -B^+ c.
// B^+ is the exact inverse when det > 1e-12 B11 B22, else the rank-one
// pseudo-inverse B / tr(B)^2 (zero when tr(B) = 0).
// ---------------------------------------------------------------------------
// Fixed-order reduction of one block's slots and the 2x2 solve; all NT
// threads of the workgroup take part.
__device__ __forceinline__ void solve_block(const Params &prm, const BlockRange &br, int ntg, int ntd,
                                            const double *__restrict__ pg, const double *__restrict__ pd,
                                            double *__restrict__ u, double *__restrict__ info,
                                            const int *__restrict__ stop)
{
    constexpr int NV = NQG + NQD;
    __shared__ double red[NT / 64][NV];
    __shared__ double tot[NV];
    // each thread sums its slots in order, then one tree over the threads;
    // the slots are read CH per thread at a time, gradient and direction
    // slots together, so their loads are in flight at once
    constexpr int CH = 4;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    {
        const double *p1 = pg + (size_t)br.g0 * ntg * NQG;
        const double *p2 = pd + (size_t)br.d0 * ntd * NQD;
        const int n1 = br.gn * ntg, n2 = br.dn * ntd;
        for (int t0 = threadIdx.x; t0 < n1 || t0 < n2; t0 += CH * NT) {
            double a[CH][NQG], b[CH][NQD];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int t = t0 + c * NT;
#pragma unroll
                for (int v = 0; v < NQG; ++v) a[c][v] = t < n1 ? p1[(size_t)t * NQG + v] : 0.0;
#pragma unroll
                for (int v = 0; v < NQD; ++v) b[c][v] = t < n2 ? p2[(size_t)t * NQD + v] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
#pragma unroll
                for (int v = 0; v < NQG; ++v) acc[v] += a[c][v];
#pragma unroll
                for (int v = 0; v < NQD; ++v) acc[NQG + v] += b[c][v];
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double sv = wave_sum_last(acc[v]);
        if (lane == 63) red[wave][v] = sv;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double sv = 0.0;
        for (int w = 0; w < NT / 64; ++w) sv += red[w][threadIdx.x];
        tot[threadIdx.x] = sv;
    }
    __syncthreads();
    // once the run has stopped nothing is written (the flag is read here,
    // not at entry, so that its load overlaps those of the slots)
    if (threadIdx.x == 0 && !(stop && *stop)) {
        // gradient pass: <g,g>, <g,dp>, <dp,dp>, then the TV curvature sums;
        // direction pass: <Hd_a,Hd_b>, then <VZ d_a, VZ d_b> (weighted by
        // 2 kappa + lambda w already when the TV is taken along z)
        const double gg = tot[0], gd = tot[1], dd = tot[2];
        const double *w = tot + 3, *h = tot + NQG, *z = tot + NQG + 3;
        const double e2 = 2.0 * prm.eta + prm.mu, k2 = prm.tv3d ? 1.0 : 2.0 * prm.kappa, lam = prm.lambda;
        double b11 = h[0] + e2 * gg + lam * w[0] + k2 * z[0];
        double b12 = h[1] - e2 * gd + lam * w[1] + k2 * z[1];
        double b22 = h[2] + e2 * dd + lam * w[2] + k2 * z[2];
        const double c1 = -gg;
        double c2 = gd;
        if (prm.method == M_GD || prm.method == M_CG) {
            // the metric L Id (Sec. 3.2): B = L D^T D over D = [-g] (Async-GD)
            // or D = [-g, dp] (Async-CG)
            const double lm = prm.lip + prm.mu;
            b11 = lm * gg;
            b12 = prm.method == M_CG ? -lm * gd : 0.0;
            b22 = prm.method == M_CG ? lm * dd : 0.0;
            if (prm.method == M_GD) c2 = 0.0;
        }
        const double det = b11 * b22 - b12 * b12, tr = b11 + b22;
        double p11, p12, p22;
        if (prm.method == M_GD) {
            // a single direction: the step -c1 / b11 (zero when g = 0)
            p11 = b11 > 0.0 ? 1.0 / b11 : 0.0;
            p12 = p22 = 0.0;
        } else if (det > 1e-12 * b11 * b22) {
            p11 = b22 / det;
            p12 = -b12 / det;
            p22 = b11 / det;
        } else if (tr > 0.0) {
            const double t2 = tr * tr;
            p11 = b11 / t2;
            p12 = b12 / t2;
            p22 = b22 / t2;
        } else {
            p11 = p12 = p22 = 0.0;
        }
        // (Async-GD: the quotient itself, -c1 / b11)
        const double u1 = prm.method == M_GD ? (b11 > 0.0 ? -c1 / b11 : 0.0) : -(p11 * c1 + p12 * c2);
        const double u2 = -(p12 * c1 + p22 * c2);
        u[2 * br.block] = u1;
        u[2 * br.block + 1] = u2;
        if (info) {
            double *o = info + 8 * br.block;
            o[0] = b11; o[1] = b12; o[2] = b22; o[3] = c1; o[4] = c2; o[5] = u1; o[6] = u2; o[7] = gg;
        }
    }
}

__global__ void __launch_bounds__(NT)
k_solve(Params prm, const BlockRange *__restrict__ brs, int ntg, int ntd, const double *__restrict__ pg,
        const double *__restrict__ pd, double *__restrict__ u, double *__restrict__ info,
        const int *__restrict__ stop)
{
    solve_block(prm, brs[blockIdx.x], ntg, ntd, pg, pd, u, info, stop);
}

// ---------------------------------------------------------------------------
// Direction pass for the block S = [z0, z0+n): with d1 = -g and d2 = dp (zero
// outside S), on output slice k
//   (H d)_k = XY_k( sum_c gz_k[c] d_{k-c} ),
// stored for the update pass, and the sums <Hd_a, Hd_b> and
// <VZ d_a, VZ d_b> (a, b in {1, 2}) of the slice, per tile.
// A workgroup takes one or two consecutive output slices k, k+1 of a block
// (a unit): their z-combines share KZ - 1 source slices, which are read once.
// ---------------------------------------------------------------------------

// Weight of the products of z differences of a block step at voxel o =
// (k, j, i): with the total variation taken along z as well (TV3) it is
// 2 kappa + lambda w, w of the current x there computed as the gradient pass
// does; otherwise 1 (the solve multiplies the plain sums by 2 kappa).
template <typename T>
__device__ __forceinline__ double zweight(const Geom &g, const Params &prm, const T *__restrict__ x, int k,
                                          int j, int i, size_t o)
{
    if (!prm.tv3d) return 1.0;
    const size_t S = (size_t)g.nx * g.ny;
    const T xv = x[o];
    const T dxv = (i < g.nx - 1) ? x[o + 1] - xv : T(0);
    const T dyv = (j < g.ny - 1) ? x[o + g.nx] - xv : T(0);
    const T dzv = (k < g.nz - 1) ? x[o + S] - xv : T(0);
    const T w = inv_sqrt(dxv * dxv + dyv * dyv + dzv * dzv + (T)(prm.delta * prm.delta));
    return 2.0 * prm.kappa + prm.lambda * (double)w;
}

// LDS passes, stores and sums of one output slice kk (direction item i) from
// its z-combined d1, d2 on the tile plus an R halo.  ONE: only d1 was
// z-combined; H d2 = H dp is the one the update pass of the block's previous
// visit formed and stored (slot i of s.hd[1]), read here for the sums, on
// the slices S +- r_z it reaches (live); the direction items below them (the
// slice under the block that the VZ sums need when r_z = 0) have H dp = 0 and
// no update item that would store it.
template <typename T, int R, int TYK, bool ONE, int E>
__device__ __forceinline__ void dirs_finish(const Geom &g, const Params &prm, const DevState<T> &s,
                                            const Item &it, int kk, size_t i, const T (&v1)[E],
                                            const T (&v2)[E], const uint32_t (&off)[E], const bool (&inb)[E],
                                            T *A1, T *A2, T *B1, double *partials, uint2 tl, const VB &vb,
                                            bool live)
{
    constexpr int NRK = TYK / (NT / TX);
    constexpr int K = 2 * R + 1, W = TX + 2 * R, H = TYK + 2 * R, N = W * H;
    constexpr int WS = vstride<T, W>();
    T *const B2 = A1;
    double *const red = reinterpret_cast<double *>(A2);
    const int z0 = it.z0, z1 = it.z0 + it.n;
    const int x0 = tl.x * TX, y0 = tl.y * TYK;
    const int tx = threadIdx.x & (TX - 1);
    const size_t S = (size_t)g.nx * g.ny;
    T wx[K], wy[K];
    load_taps<T, R>(wx, s.gx + (size_t)kk * K);
    load_taps<T, R>(wy, s.gy + (size_t)kk * K);
    const __amdgpu_buffer_rsrc_t o1 = buf_of(s.hd[0] + i * S, S), o2 = buf_of(s.hd[1] + i * S, S);
    T h1[NRK], h2[NRK];
    if constexpr (ONE) {
        // H dp of the outputs, loaded first so that the LDS passes hide it
#pragma unroll
        for (int e = 0; e < NRK; ++e) {
            const int j = y0 + out_row<NRK>(e), ii = x0 + tx;
            const uint32_t o = (ii < g.nx && j < g.ny) ? (uint32_t)(j * g.nx + ii) * (uint32_t)sizeof(T) : 0u;
            const T v = ldbuf<T>(o2, o);
            h2[e] = live ? v : T(0);
        }
    }
#pragma unroll
    for (int qq = 0; qq < E; ++qq) {
        const int e = threadIdx.x + qq * NT;
        if (N % NT != 0 && e >= N) break;
        A1[lds_at<W, WS>(e)] = inb[qq] ? v1[qq] : T(0);
        if constexpr (!ONE) A2[lds_at<W, WS>(e)] = inb[qq] ? v2[qq] : T(0);
    }
    __syncthreads();
    xpass4<T, R, H, false>(A1, B1, wx);
    __syncthreads();
    if constexpr (!ONE) {
        xpass4<T, R, H, false>(A2, B2, wx);
        __syncthreads();
    }
    ypass_out<T, R, TX, R, false, NRK>(B1, h1, wy);
    if constexpr (!ONE) ypass_out<T, R, TX, R, false, NRK>(B2, h2, wy);
    {
        // stored for the update pass, which combines them with the step
        // coefficients instead of blurring the new step again
#pragma unroll
        for (int e = 0; e < NRK; ++e) {
            const int j = y0 + out_row<NRK>(e), ii = x0 + tx;
            if (ii >= g.nx || j >= g.ny) continue;
            const uint32_t o = (uint32_t)(j * g.nx + ii) * (uint32_t)sizeof(T);
            stbuf(o1, o, h1[e]);
            if constexpr (!ONE) stbuf(o2, o, h2[e]);
        }
    }
    double qs[NQD];
#pragma unroll
    for (int v = 0; v < NQD; ++v) qs[v] = 0.0;
    const bool ink = (kk >= z0 && kk < z1);
    const bool zsums = prm.kappa != 0.0 || prm.tv3d;
    const bool zterm = zsums && kk >= z0 - 1 && kk < z1 && kk < g.nz - 1;
    const T *__restrict__ gg = s.g;
    const T *__restrict__ dpv = s.dp[0];
#pragma unroll
    for (int e = 0; e < NRK; ++e) {
        const int j = y0 + out_row<NRK>(e), ii = x0 + tx;
        // every row of the tile without a branch: outputs outside the slice
        // add exact zeros
        const bool ok = ii < g.nx && j < g.ny;
        const double a = ok ? (double)h1[e] : 0.0, b = ok ? (double)h2[e] : 0.0;
        qs[0] += a * a;
        qs[1] += a * b;
        qs[2] += b * b;
        if (zterm && ok) {
            // VZ d at slice kk: d_{kk+1} - d_kk with d zero outside S
            const size_t o = vidx(g, kk, j, ii);
            double z1v = 0.0, z2v = 0.0;
            if (kk + 1 >= z0 && kk + 1 < z1) {
                z1v -= (double)gg[o + S];
                z2v += (double)dpv[o + S];
            }
            if (ink) {
                z1v += (double)gg[o];
                z2v -= (double)dpv[o];
            }
            const double c = zweight(g, prm, s.x, kk, j, ii, o);
            qs[3] += c * z1v * z1v;
            qs[4] += c * z1v * z2v;
            qs[5] += c * z2v * z2v;
        }
    }
    // without a VZ term the last three sums are zero
    wg_reduce_store<NQD>(qs, red, partials + ((i * vb.gy + tl.y) * vb.gx + tl.x) * NQD,
                         zsums ? NQD : 3);
}

template <typename T, int KZ, int R, int TYK, bool ONE = false>
__device__ __forceinline__ void dirs_body(const VB vb, Geom g, Params prm, DevState<T> s,
                                          const Item *__restrict__ units, double *__restrict__ partials)
{
    constexpr int RZ = KZ / 2;
    constexpr int W = TX + 2 * R, H = TYK + 2 * R;
    // the x pass of d2 is written over the z-combine of d1, and the
    // reduction of the inner products over the z-combine of d2 (three tiles,
    // not four: more workgroups fit a compute unit's LDS); ONE has no d2
    // tile, only room for the reduction
    constexpr int WS = vstride<T, W>();
    constexpr int NRED = (NT / 64) * NQD * (int)(sizeof(double) / sizeof(T));
    __shared__ __align__(16) T A1[padded<WS, H>()];
    __shared__ __align__(16) T A2[ONE ? NRED : padded<WS, H>()];
    __shared__ __align__(16) T B1[padded<TX, H>()];
    static_assert(padded<TX, H>() <= padded<WS, H>(), "x pass of d2 must fit the d1 tile");
    static_assert(NRED <= padded<WS, H>(), "reduction must fit");

    // slice k of the block [z0, z0 + n): direction items h0 and, when hn is
    // 2, h0 + 1 (slice k + 1)
    // tiles in the XCD-aware order within the slice; slices in plain order,
    // which keeps the same tile of consecutive slices (sharing KZ - 1
    // source slices) on one XCD close in time (the whole-grid order of the
    // update pass would spread them out and lose that reuse)
    const uint2 tl = xcd_slice_tile(vb);
    const Item it = units[vb.z];
    if (s.stop && *s.stop) return;  // read with the unit, not before it
    const int k = it.k, z0 = it.z0, z1 = it.z0 + it.n;
    const bool two = it.hn > 1;
    const int x0 = tl.x * TX, y0 = tl.y * TYK;
    const size_t S = (size_t)g.nx * g.ny;
    const T *__restrict__ gg = s.g;
    const T *__restrict__ dpv = s.dp[0];
    const T *wz0 = s.gz + (size_t)k * KZ;
    const T *wz1 = s.gz + (size_t)(two ? k + 1 : k) * KZ;

    // z-combines of d1 and d2 for slices k (a) and k + 1 (b) on the tile plus
    // an R halo: source slice sl = k - RZ + t, tap k - sl of slice k and
    // tap k + 1 - sl of slice k + 1 (sources in decreasing z, the order of a
    // single slice's sum)
    Region<W, H, R, R> rg(g, x0, y0);
    T a1[rg.E], a2[rg.E], b1[rg.E], b2[rg.E];
    uint32_t bo[rg.E];
#pragma unroll
    for (int qq = 0; qq < rg.E; ++qq) {
        a1[qq] = a2[qq] = b1[qq] = b2[qq] = 0;
        bo[qq] = rg.off[qq] * (uint32_t)sizeof(T);
    }
#pragma unroll
    for (int t = KZ; t >= 0; --t) {
        const int sl = k - RZ + t;
        if (sl < z0 || sl >= z1 || (t == KZ && !two)) continue;
        const T wa = t < KZ ? wz0[KZ - 1 - t] : T(0);
        const T wb = t > 0 && two ? wz1[KZ - t] : T(0);
        const __amdgpu_buffer_rsrc_t gs = buf_of(gg + (size_t)sl * S, S), ds = buf_of(dpv + (size_t)sl * S, S);
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const T gv = ldbuf<T>(gs, bo[qq]);
            const T dv = ONE ? T(0) : ldbuf<T>(ds, bo[qq]);
            if (t < KZ) {
                a1[qq] -= wa * gv;
                if constexpr (!ONE) a2[qq] += wa * dv;
            }
            if (t > 0) {
                b1[qq] -= wb * gv;
                if constexpr (!ONE) b2[qq] += wb * dv;
            }
        }
    }
    dirs_finish<T, R, TYK, ONE>(g, prm, s, it, k, (size_t)it.h0, a1, a2, rg.off, rg.inb, A1, A2, B1, partials, tl,
                                vb, k >= z0 - RZ);
    if (two) {
        __syncthreads();  // the reduction of slice k read A2
        dirs_finish<T, R, TYK, ONE>(g, prm, s, it, k + 1, (size_t)it.h0 + 1, b1, b2, rg.off, rg.inb, A1, A2, B1,
                                    partials, tl, vb, k + 1 >= z0 - RZ);
    }
}

template <typename T, int KZ, int R, int TYK, bool ONE>
__global__ void __launch_bounds__(NT)
k_dirs(Geom g, Params prm, DevState<T> s, const Item *__restrict__ units, double *__restrict__ partials)
{
    dirs_body<T, KZ, R, TYK, ONE>(vb_native(), g, prm, s, units, partials);
}

// ---------------------------------------------------------------------------
// Update pass, one slice m per item, from the direction pass's stored
// H d1, H d2 (d1 = -g, d2 = dp on the block S, zero elsewhere):
//   (H d')_m = sum over the item's pairs (slot, b) of u1_b (H d1)_slot + u2_b (H d2)_slot,
//   q_m += XY^T_m (H d')_m,
//   and for m in the item's own block: d'_m = -u1 g_m + u2 dp_m, x_m += d'_m,
//   dp[1]_m = d'_m.
// A coloured group has one pair per item (the blocks of a colour have
// disjoint S +- r_z); a round has every block whose S +- r_z holds m (the
// steps have disjoint supports, so H of their sum is the sum of their H).
// H d' is read on the tile plus an R halo (zero outside the slice: the
// adjoint blur sees zero padding), then blurred back by the adjoint x and y
// passes of slice m.  Previous steps are read from dp[0] and written to
// dp[1], so a workgroup never sees a half-updated step.  When s.hdw is set,
// each pair's H d' on the tile is also stored in its slot there: the H dp of
// the block's next visit, so that its direction pass blurs only d1.
// ---------------------------------------------------------------------------
template <typename T, int R, int TYK, bool MULTI, bool STREAM = false>
__device__ __forceinline__ void update_body(const VB vb, Geom g, DevState<T> s, const Item *__restrict__ items,
                                            const int2 *__restrict__ pairs, const double *__restrict__ u, int assign)
{
    constexpr int NRK = TYK / (NT / TX);
    constexpr int K = 2 * R + 1;
    constexpr int W2 = TX + 2 * R, H2 = TYK + 2 * R, WS2 = vstride<T, W2>();
    __shared__ __align__(16) T A[padded<WS2, H2>()];
    __shared__ __align__(16) T B[padded<TX, H2>()];

    const uint3 bk = xcd_block(vb);
    const Item it = items[bk.z];
    if (s.stop && *s.stop) return;  // read with the item, not before it
    const int m = it.k;
    const int x0 = bk.x * TX, y0 = bk.y * TYK;
    const int tx = threadIdx.x & (TX - 1);
    const size_t S = (size_t)g.nx * g.ny;
    T wx[K], wy[K];
    load_taps<T, R>(wx, s.gx + (size_t)m * K);
    load_taps<T, R>(wy, s.gy + (size_t)m * K);
    // the outputs' q, and on the block x, dp and g, are loaded first so that
    // their latency overlaps the loads of H d' (no pass of this launch writes
    // H d1 or H d2)
    // assign: s.q receives XY^T_m (H d')_m itself, and x, dp are left alone
    // (the majorant applied to a block vector, Async-MM's inner solve)
    const bool ins = !assign && (m >= it.z0 && m < it.z0 + it.n);
    const __amdgpu_buffer_rsrc_t qs = buf_of(s.q + (size_t)m * S, S), xs = buf_of(s.x + (size_t)m * S, S);
    const __amdgpu_buffer_rsrc_t ds = buf_of(s.dp[0] + (size_t)m * S, S), gs = buf_of(s.g + (size_t)m * S, S);
    T qv[NRK], xv[NRK], dv[NRK], gv[NRK];
#pragma unroll
    for (int e = 0; e < NRK; ++e) {
        const int j = y0 + out_row<NRK>(e), i = x0 + tx;
        const uint32_t o = (i < g.nx && j < g.ny) ? (uint32_t)(j * g.nx + i) * (uint32_t)sizeof(T) : 0u;
        qv[e] = assign ? T(0) : ldbuf<T>(qs, o);
        xv[e] = dv[e] = gv[e] = 0;
        if (ins) {
            xv[e] = ldbuf<T>(xs, o);
            dv[e] = ldbuf<T>(ds, o);
            gv[e] = ldbuf<T>(gs, o);
        }
    }
    {
        Region<W2, H2, R, R> rg(g, x0, y0);
        T v[rg.E];
        uint32_t bo[rg.E];
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            v[qq] = 0;
            bo[qq] = rg.off[qq] * (uint32_t)sizeof(T);
        }
        // a round: the tile's own elements of the region (not its halo),
        // where each pair's H d' is stored for the next visit (a colour has
        // one pair, whose H d' is stored from the LDS tile below)
        bool own[MULTI ? rg.E : 1];
        if constexpr (MULTI) {
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) {
                const int e = threadIdx.x + qq * NT;
                const int jj = e / W2, ii = e - jj * W2;
                own[qq] = rg.inb[qq] && jj >= R && jj < R + TYK && ii >= R && ii < R + TX;
            }
        }
        // sources two at a time, so that the loads of both are in flight
        // together (a round has several per slice; a colour has one, and
        // its instance carries no code for more)
        int p = 0;
        for (; MULTI && p + 1 < it.hn; p += 2) {
            const int2 pa = pairs[it.h0 + p], pb = pairs[it.h0 + p + 1];
            const T a1 = (T)u[2 * pa.y], a2 = (T)u[2 * pa.y + 1];
            const T b1 = (T)u[2 * pb.y], b2 = (T)u[2 * pb.y + 1];
            const __amdgpu_buffer_rsrc_t ha1 = buf_of(s.hd[0] + (size_t)pa.x * S, S);
            const __amdgpu_buffer_rsrc_t ha2 = buf_of(s.hd[1] + (size_t)pa.x * S, S);
            const __amdgpu_buffer_rsrc_t hb1 = buf_of(s.hd[0] + (size_t)pb.x * S, S);
            const __amdgpu_buffer_rsrc_t hb2 = buf_of(s.hd[1] + (size_t)pb.x * S, S);
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) {
                const T xa1 = ldbuf<T>(ha1, bo[qq]), xa2 = ldbuf<T>(ha2, bo[qq]);
                const T xb1 = ldbuf<T>(hb1, bo[qq]), xb2 = ldbuf<T>(hb2, bo[qq]);
                const T wa = a1 * xa1 + a2 * xa2, wb = b1 * xb1 + b2 * xb2;
                v[qq] += wa;
                v[qq] += wb;
                if (s.hdw && own[qq]) {
                    stbuf(buf_of(s.hdw + (size_t)pa.x * S, S), bo[qq], wa);
                    stbuf(buf_of(s.hdw + (size_t)pb.x * S, S), bo[qq], wb);
                }
            }
        }
        if (p < it.hn) {
            // the first pair is carried by the item itself
            const int2 pr = p == 0 ? int2{it.ps, it.pb} : pairs[it.h0 + p];
            const T c1 = (T)u[2 * pr.y], c2 = (T)u[2 * pr.y + 1];
            const __amdgpu_buffer_rsrc_t h1 = buf_of(s.hd[0] + (size_t)pr.x * S, S);
            const __amdgpu_buffer_rsrc_t h2 = buf_of(s.hd[1] + (size_t)pr.x * S, S);
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) {
                const T w = c1 * ldbuf<T>(h1, bo[qq]) + c2 * ldbuf<T>(h2, bo[qq]);
                v[qq] += w;
                if constexpr (MULTI) {
                    if (s.hdw && own[qq]) stbuf(buf_of(s.hdw + (size_t)pr.x * S, S), bo[qq], w);
                }
            }
        }
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const int e = threadIdx.x + qq * NT;
            if (rg.N % NT != 0 && e >= rg.N) break;
            A[lds_at<W2, WS2>(e)] = rg.inb[qq] ? v[qq] : T(0);
        }
    }
    // x and dp of this slice are read by no other workgroup: written now,
    // which frees their registers for the blur passes
    if (ins) {
        const T u1 = (T)u[2 * it.block], u2 = (T)u[2 * it.block + 1];
        const __amdgpu_buffer_rsrc_t xo = buf_of(s.x + (size_t)m * S, S), dpo = buf_of(s.dp[1] + (size_t)m * S, S);
#pragma unroll
        for (int e = 0; e < NRK; ++e) {
            const int j = y0 + out_row<NRK>(e), i = x0 + tx;
            if (i >= g.nx || j >= g.ny) continue;
            const uint32_t o = (uint32_t)(j * g.nx + i) * (uint32_t)sizeof(T);
            const T d = u2 * dv[e] - u1 * gv[e];
            stbuf<STREAM>(xo, o, xv[e] + d);
            stbuf<STREAM>(dpo, o, d);
        }
    }
    __syncthreads();
    if (!MULTI && s.hdw) {
        // the pair's H d' on the tile (the next visit's H dp), from the LDS
        // tile in rows of 64 lanes
        const __amdgpu_buffer_rsrc_t ho = buf_of(s.hdw + (size_t)it.ps * S, S);
#pragma unroll
        for (int e = 0; e < NRK; ++e) {
            const int j = y0 + out_row<NRK>(e), i = x0 + tx;
            if (i >= g.nx || j >= g.ny) continue;
            stbuf<STREAM>(ho, (uint32_t)(j * g.nx + i) * (uint32_t)sizeof(T), A[(out_row<NRK>(e) + R) * WS2 + tx + R]);
        }
    }
    xpass4<T, R, H2, true>(A, B, wx);
    __syncthreads();
    T v[NRK];
    ypass_out<T, R, TX, R, true, NRK>(B, v, wy);
    const __amdgpu_buffer_rsrc_t qo = buf_of(s.q + (size_t)m * S, S);
#pragma unroll
    for (int e = 0; e < NRK; ++e) {
        const int j = y0 + out_row<NRK>(e), i = x0 + tx;
        if (i >= g.nx || j >= g.ny) continue;
        stbuf<STREAM>(qo, (uint32_t)(j * g.nx + i) * (uint32_t)sizeof(T), qv[e] + v[e]);
    }
}

// STREAM: the instance whose volume stores carry the non-temporal hint (s.nt)
template <typename T, int R, int TYK, bool MULTI, bool STREAM>
__global__ void __launch_bounds__(NT)
k_update(Geom g, DevState<T> s, const Item *__restrict__ items, const int2 *__restrict__ pairs,
         const double *__restrict__ u, int assign)
{
    update_body<T, R, TYK, MULTI, STREAM>(vb_native(), g, s, items, pairs, u, assign);
}

// ---------------------------------------------------------------------------
// Refresh of the blurred residual, one slice m per item:
//   q_m = XY^T_m (H src - y)_m.
// (H src)_m is formed on the tile plus an R halo (z-combine on a 2R halo, x
// and y passes), zeroed outside the slice, then blurred back by the adjoint
// x and y passes of slice m.
// ---------------------------------------------------------------------------
template <typename T, int KZ, int R, int TYK>
__global__ void __launch_bounds__(NT)
k_refresh(Geom g, DevState<T> s, const T *__restrict__ src, T *__restrict__ qout,
          const Item *__restrict__ items)
{
    constexpr int NRK = TYK / (NT / TX);
    constexpr int RZ = KZ / 2, K = 2 * R + 1;
    constexpr int W1 = TX + 4 * R, H1 = TYK + 4 * R;  // z-combined source, 2R halo
    constexpr int W2 = TX + 2 * R, H2 = TYK + 2 * R;  // H src - y, R halo
    constexpr int WS2 = vstride<T, W2>();
    static_assert(padded<W1, H1>() >= WS2 * H2, "H src - y must fit the source tile");
    __shared__ __align__(16) T A[padded<W1, H1>()];  // z-combined source, later H src - y
    __shared__ __align__(16) T B[padded<W2, H1>()];  // forward x pass, later adjoint x pass

    const Item it = items[blockIdx.z];
    if (s.stop && *s.stop) return;  // read with the item, not before it
    const int m = it.k;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TYK;
    const int tx = threadIdx.x & (TX - 1);
    const size_t S = (size_t)g.nx * g.ny;
    const T *wz = s.gz + (size_t)m * KZ;
    T wx[K], wy[K];
    load_taps<T, R>(wx, s.gx + (size_t)m * K);
    load_taps<T, R>(wy, s.gy + (size_t)m * K);

    // 1. z-combine of the source on the tile plus a 2R halo
    {
        Region<W1, H1, 2 * R, 2 * R> rg(g, x0, y0);
        T v[rg.E];
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) v[qq] = 0;
#pragma unroll
        for (int c = -RZ; c <= RZ; ++c) {
            const int sl = min(max(m - c, 0), g.nz - 1);  // weight 0 past the volume
            const T wv = (m - c == sl) ? wz[c + RZ] : T(0);
            const T *ss = src + (size_t)sl * S;
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) v[qq] += wv * ldo(ss, rg.off[qq]);
        }
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) A[threadIdx.x + qq * NT] = rg.inb[qq] ? v[qq] : T(0);
    }
    // the data term is needed on the R halo; load it early
    Region<W2, H2, R, R> r2(g, x0, y0);
    T yv[r2.E];
    {
        const T *ys = s.y + (size_t)m * S;
#pragma unroll
        for (int qq = 0; qq < r2.E; ++qq) yv[qq] = ldo(ys, r2.off[qq]);
    }
    __syncthreads();
    // 2. forward x pass: all H1 rows, the W2 columns of the R-halo tile
    xpass<T, R, W1, W2, H1, R, false>(A, B, wx);
    __syncthreads();
    // 3. forward y pass on the R-halo tile into A (H src - y), zero outside the slice
#pragma unroll
    for (int qq = 0; qq < r2.E; ++qq) {
        const int e = threadIdx.x + qq * NT;
        if (r2.N % NT != 0 && e >= r2.N) break;
        const int r = e / W2;
        const int c = e - r * W2;
        const T *col = B + (r + R) * W2 + c;
        T acc = 0;
#pragma unroll
        for (int b = -R; b <= R; ++b) acc += wy[b + R] * col[-b * W2];
        A[r * WS2 + c] = r2.inb[qq] ? acc - yv[qq] : T(0);
    }
    __syncthreads();
    // 4. adjoint x pass over the R-halo rows into B
    xpass4<T, R, H2, true>(A, B, wx);
    __syncthreads();
    // 5. adjoint y pass into registers
    T v[NRK];
    ypass_out<T, R, TX, R, true, NRK>(B, v, wy);
#pragma unroll
    for (int e = 0; e < NRK; ++e) {
        const int j = y0 + out_row<NRK>(e), i = x0 + tx;
        if (i >= g.nx || j >= g.ny) continue;
        qout[vidx(g, m, j, i)] = v[e];
    }
}

// ---------------------------------------------------------------------------
// out_k = (H in)_k - sub_k per item; optional per-slot sums of out^2.
// ---------------------------------------------------------------------------
template <typename T, int KZ, int R, int TYK>
__global__ void __launch_bounds__(NT)
k_H(Geom g, DevState<T> s, const T *__restrict__ in, const T *__restrict__ sub, T *__restrict__ out,
    const Item *__restrict__ items, double *__restrict__ partials)
{
    constexpr int NRK = TYK / (NT / TX);
    constexpr int RZ = KZ / 2, K = 2 * R + 1;
    constexpr int W = TX + 2 * R, H = TYK + 2 * R, WS = vstride<T, W>();
    __shared__ __align__(16) T A[padded<WS, H>()];
    __shared__ __align__(16) T B[padded<TX, H>()];
    __shared__ double red[NT / 64];
    const Item it = items[blockIdx.z];
    if (s.stop && *s.stop) return;  // read with the item, not before it
    const int k = it.k;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TYK;
    const int tx = threadIdx.x & (TX - 1);
    const size_t S = (size_t)g.nx * g.ny;
    const T *wz = s.gz + (size_t)k * KZ;
    T wx[K], wy[K];
    load_taps<T, R>(wx, s.gx + (size_t)k * K);
    load_taps<T, R>(wy, s.gy + (size_t)k * K);
    {
        Region<W, H, R, R> rg(g, x0, y0);
        T v[rg.E];
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) v[qq] = 0;
#pragma unroll
        for (int c = -RZ; c <= RZ; ++c) {
            const int sl = min(max(k - c, 0), g.nz - 1);  // weight 0 past the volume
            const T wv = (k - c == sl) ? wz[c + RZ] : T(0);
            const T *ss = in + (size_t)sl * S;
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) v[qq] += wv * ldo(ss, rg.off[qq]);
        }
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const int e = threadIdx.x + qq * NT;
            if (rg.N % NT != 0 && e >= rg.N) break;
            A[lds_at<W, WS>(e)] = rg.inb[qq] ? v[qq] : T(0);
        }
    }
    __syncthreads();
    xpass4<T, R, H, false>(A, B, wx);
    __syncthreads();
    T h[NRK];
    ypass_out<T, R, TX, R, false, NRK>(B, h, wy);
    double ss[1] = {0.0};
#pragma unroll
    for (int e = 0; e < NRK; ++e) {
        const int j = y0 + out_row<NRK>(e), i = x0 + tx;
        if (i < g.nx && j < g.ny) {
            const size_t o = vidx(g, k, j, i);
            const T v = sub ? h[e] - sub[o] : h[e];
            out[o] = v;
            ss[0] += (double)v * (double)v;
        }
    }
    if (partials) wg_reduce_store<1>(ss, red, partials + slot_of(vb_native()));
}

// ---------------------------------------------------------------------------
// out_m = XY^T_m in_m per item (adjoint in-slice blur with slice m's factors).
// ---------------------------------------------------------------------------
template <typename T, int R, int TYK>
__global__ void __launch_bounds__(NT)
k_blurT(Geom g, DevState<T> s, const T *__restrict__ in, T *__restrict__ out,
        const Item *__restrict__ items)
{
    constexpr int NRK = TYK / (NT / TX);
    constexpr int K = 2 * R + 1;
    constexpr int W = TX + 2 * R, H = TYK + 2 * R, WS = vstride<T, W>();
    __shared__ __align__(16) T A[padded<WS, H>()];
    __shared__ __align__(16) T B[padded<TX, H>()];
    const Item it = items[blockIdx.z];
    const int m = it.k;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TYK;
    const int tx = threadIdx.x & (TX - 1);
    T wx[K], wy[K];
    load_taps<T, R>(wx, s.gx + (size_t)m * K);
    load_taps<T, R>(wy, s.gy + (size_t)m * K);
    {
        Region<W, H, R, R> rg(g, x0, y0);
        const T *im = in + (size_t)m * g.nx * g.ny;
        T v[rg.E];
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) v[qq] = ldo(im, rg.off[qq]);
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const int e = threadIdx.x + qq * NT;
            if (rg.N % NT != 0 && e >= rg.N) break;
            A[lds_at<W, WS>(e)] = rg.inb[qq] ? v[qq] : T(0);
        }
    }
    __syncthreads();
    xpass4<T, R, H, true>(A, B, wx);
    __syncthreads();
    T v[NRK];
    ypass_out<T, R, TX, R, true, NRK>(B, v, wy);
#pragma unroll
    for (int e = 0; e < NRK; ++e) {
        const int j = y0 + out_row<NRK>(e), i = x0 + tx;
        if (i < g.nx && j < g.ny) out[vidx(g, m, j, i)] = v[e];
    }
}

__global__ void __launch_bounds__(NT)
k_sum(const double *__restrict__ partials, int nslot, int nq, double *__restrict__ out)
{
    __shared__ double red[NT];
    for (int v = 0; v < nq; ++v) {
        double sv = 0.0;
        for (int t = threadIdx.x; t < nslot; t += NT) sv += partials[(size_t)t * nq + v];
        red[threadIdx.x] = sv;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[v] = red[0];
        __syncthreads();
    }
}

// Stop test on the device: ||grad f|| from the evaluation slots (fixed-order
// sum), recorded in *gnorm; when it is at most thr, *stop is raised and the
// sweep number recorded, and every later pass of the run returns without
// writing.
__global__ void __launch_bounds__(NT)
k_check(const double *__restrict__ partials, int nslot, double thr, int sweep, int *stop,
        int *stop_sweep, double *gnorm)
{
    __shared__ double red[NT];
    if (*stop) return;
    double sv = 0.0;
    for (int t = threadIdx.x; t < nslot; t += NT) sv += partials[(size_t)t * NQE];
    red[threadIdx.x] = sv;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double gn = sqrt(red[0]);
        *gnorm = gn;
        if (gn <= thr) {
            *stop = 1;
            *stop_sweep = sweep;
        }
    }
}

// ---------------------------------------------------------------------------
// General per-depth kernels (dense PSF).  The kernel of output slice k is a
// (2 rz + 1) x (2R + 1) x (2R + 1) table P_k[c][b][a] (zero-padded in-slice
// to the radius R of the kernel instance; pk is [nz][kz][2R+1][2R+1]):
//   forward  (H x)_k[j][i]   = sum_{c,b,a} P_k[c][b][a]     x_{k-c}[j-b][i-a],
//   adjoint  (H^T r)_s[j][i] = sum_{c,b,a} P_{s+c}[c][b][a] r_{s+c}[j+b][i+a].
// A workgroup computes a TX x TYD output tile of one slice (TYD = 16 or 32,
// the direction-pass tile height of the problem): for each source
// slice in turn, the source tile plus an R halo is staged in LDS (the next
// source's loads are in flight while the current one is consumed), and each
// thread slides the 2D stencil over NRD consecutive rows of its column: for
// each tap column it reads the NRD + 2R values of the column once.
// ---------------------------------------------------------------------------

template <typename T, int R, int NCH, bool ADJ, int NRD>
__device__ __forceinline__ void dense_accumulate(const T *L, int ldw, const T *__restrict__ w,
                                                 T (&acc)[NCH][NRD], int nch_stride)
{
    constexpr int K = 2 * R + 1, NV = NRD + 2 * R;
    const int tx = threadIdx.x & (TX - 1);
    const int r0 = (int)(threadIdx.x / TX) * NRD;
    // one tap column at a time (unrolling this loop as well would hold the
    // columns of several taps in registers)
#pragma unroll 1
    for (int a = -R; a <= R; ++a) {
        // forward: column tx + R - a, rows r0 + e + R - b; adjoint: + a, + b
        const int col = tx + R + (ADJ ? a : -a);
        T v[NCH][NV];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int t = 0; t < NV; ++t) v[ch][t] = L[ch * nch_stride + (r0 + t) * ldw + col];
#pragma unroll
        for (int b = -R; b <= R; ++b) {
            const T wv = w[(b + R) * K + (a + R)];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int e = 0; e < NRD; ++e) acc[ch][e] += wv * v[ch][e + R + (ADJ ? b : -b)];
        }
    }
}

template <typename T, int R, int NCH, bool ADJ, int TYD>
__global__ void __launch_bounds__(NT)
k_dense(Geom g, Params prm, DevState<T> s, const T *__restrict__ pk, const T *__restrict__ in,
        const T *__restrict__ sub, T *__restrict__ out, const Item *__restrict__ items, int mode,
        double *__restrict__ partials, int nsplit)
{
    constexpr int NRD = TYD / (NT / TX);  // rows per thread
    constexpr int K = 2 * R + 1, W = TX + 2 * R, H = TYD + 2 * R;
    constexpr int LT = padded<W, H>();
    __shared__ T L[NCH * LT];
    __shared__ double red[(NT / 64) * NQD];
    // nsplit > 1 (adjoint only): workgroup z = item nsplit + part, each part
    // a contiguous share of the item's source slices, written to the plane
    // out + part (number of items) S + item S, added in order by the reader
    const int ii = nsplit > 1 ? (int)blockIdx.z / nsplit : (int)blockIdx.z;
    const int part = nsplit > 1 ? (int)blockIdx.z - ii * nsplit : 0;
    const Item it = items[ii];
    if (s.stop && *s.stop) return;  // read with the item, not before it
    const int k = it.k;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TYD;
    const int tx = threadIdx.x & (TX - 1);
    const int rz = g.rz, kz = 2 * g.rz + 1;
    const size_t S = (size_t)g.nx * g.ny;
    const bool dirs = (mode == DM_DIRS);
    // source slices: forward sl = k - c, adjoint sl = k + c, c in [-rz, rz],
    // inside the volume, and for the direction pass inside the item's block
    const int lo = dirs ? it.z0 : 0, hi = dirs ? it.z0 + it.n : g.nz;
    const int a0 = max(k - rz, lo), a1 = min(k + rz + 1, hi);
    const int len = max(a1 - a0, 0);
    const int s0 = a0 + (len * part) / nsplit, s1 = a0 + (len * (part + 1)) / nsplit;  // [s0, s1)
    Region<W, H, R, R> rg(g, x0, y0);
    T st[NCH][rg.E];
    auto fetch = [&](int sl) {
        const T *p0 = dirs ? s.g + (size_t)sl * S : in + (size_t)sl * S;
        const T *p1 = s.dp[0] + (size_t)sl * S;
#pragma unroll
        for (int qq = 0; qq < rg.E; ++qq) {
            const T v0 = ldo(p0, rg.off[qq]);
            st[0][qq] = rg.inb[qq] ? (dirs ? -v0 : v0) : T(0);
            if constexpr (NCH > 1) {
                const T v1 = ldo(p1, rg.off[qq]);
                st[1][qq] = rg.inb[qq] ? v1 : T(0);
            }
        }
    };
    T acc[NCH][NRD];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int e = 0; e < NRD; ++e) acc[ch][e] = 0;
    if (s0 < s1) fetch(s0);
    for (int sl = s0; sl < s1; ++sl) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int qq = 0; qq < rg.E; ++qq) L[ch * LT + threadIdx.x + qq * NT] = st[ch][qq];
        __syncthreads();
        if (sl + 1 < s1) fetch(sl + 1);  // in flight while this slice is consumed
        // forward: tap c = k - sl of output slice k; adjoint: tap c = sl - k of source slice sl
        const T *w = ADJ ? pk + ((size_t)sl * kz + (sl - k + rz)) * K * K
                         : pk + ((size_t)k * kz + (k - sl + rz)) * K * K;
        dense_accumulate<T, R, NCH, ADJ, NRD>(L, W, w, acc, LT);
        __syncthreads();
    }

    double qs[NQD];
#pragma unroll
    for (int v = 0; v < NQD; ++v) qs[v] = 0.0;
    const int r0 = (int)(threadIdx.x / TX) * NRD;
    if (dirs) {
        T *o1 = s.hd[0] + (size_t)blockIdx.z * S, *o2 = s.hd[1] + (size_t)blockIdx.z * S;
        const int z0 = it.z0, z1 = it.z0 + it.n;
        const bool ink = (k >= z0 && k < z1);
        const bool zterm = (prm.kappa != 0.0 || prm.tv3d) && k >= z0 - 1 && k < z1 && k < g.nz - 1;
#pragma unroll
        for (int e = 0; e < NRD; ++e) {
            const int j = y0 + r0 + e, i = x0 + tx;
            if (i >= g.nx || j >= g.ny) continue;
            const size_t o = (size_t)j * g.nx + i;
            o1[o] = acc[0][e];
            o2[o] = acc[NCH - 1][e];
            const double a = (double)acc[0][e], b = (double)acc[NCH - 1][e];
            qs[0] += a * a;
            qs[1] += a * b;
            qs[2] += b * b;
            if (zterm) {
                // VZ d at slice k: d_{k+1} - d_k with d zero outside S
                const size_t ov = (size_t)k * S + o;
                double z1v = 0.0, z2v = 0.0;
                if (k + 1 >= z0 && k + 1 < z1) {
                    z1v -= (double)s.g[ov + S];
                    z2v += (double)s.dp[0][ov + S];
                }
                if (ink) {
                    z1v += (double)s.g[ov];
                    z2v -= (double)s.dp[0][ov];
                }
                const double c = zweight(g, prm, s.x, k, j, i, ov);
                qs[3] += c * z1v * z1v;
                qs[4] += c * z1v * z2v;
                qs[5] += c * z2v * z2v;
            }
        }
        wg_reduce_store<NQD>(qs, red, partials + slot_of(vb_native()) * NQD);
        return;
    }
    const size_t base = nsplit > 1 ? ((size_t)part * (gridDim.z / nsplit) + ii) * S : (size_t)k * S;
#pragma unroll
    for (int e = 0; e < NRD; ++e) {
        const int j = y0 + r0 + e, i = x0 + tx;
        if (i >= g.nx || j >= g.ny) continue;
        const size_t o = (size_t)j * g.nx + i;
        const T v = sub ? acc[0][e] - sub[(size_t)k * S + o] : acc[0][e];
        out[base + o] = v;
        qs[0] += (double)v * (double)v;
    }
    if (partials) {
        double q1[1] = {qs[0]};
        wg_reduce_store<1>(q1, red, partials + slot_of(vb_native()));
    }
}

// Update pass of the dense mode, where the maintained vector is the residual
// r = Hx - y itself: per item (slice m),
//   r_m += sum over the item's pairs (slot, b) of u1_b (H d1)_slot + u2_b (H d2)_slot,
//   and for m in the item's own block: d' = -u1 g + u2 dp, x += d', dp[1] = d'.
template <typename T>
__global__ void __launch_bounds__(NT)
k_dense_update(Geom g, DevState<T> s, const Item *__restrict__ items, const int2 *__restrict__ pairs,
               const double *__restrict__ u)
{
    const Item it = items[blockIdx.z];
    if (s.stop && *s.stop) return;  // read with the item, not before it
    const int m = it.k;
    const size_t S = (size_t)g.nx * g.ny;
    const bool ins = (m >= it.z0 && m < it.z0 + it.n);
    const T u1 = ins ? (T)u[2 * it.block] : T(0), u2 = ins ? (T)u[2 * it.block + 1] : T(0);
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < S; e += (size_t)gridDim.x * NT) {
        const size_t o = (size_t)m * S + e;
        T acc = s.q[o];
        for (int p = 0; p < it.hn; ++p) {
            const int2 pr = pairs[it.h0 + p];
            acc += (T)u[2 * pr.y] * s.hd[0][(size_t)pr.x * S + e] + (T)u[2 * pr.y + 1] * s.hd[1][(size_t)pr.x * S + e];
        }
        s.q[o] = acc;
        if (ins) {
            const T d = u2 * s.dp[0][o] - u1 * s.g[o];
            s.x[o] += d;
            s.dp[1][o] = d;
        }
    }
}

// ---------------------------------------------------------------------------
// Async-MM (Sec. 3.2, "Ablation study and comparative analysis"): the
// Worker's direction d' = -A_S(x)^{-1} grad_S f, the half-quadratic block
// majorant inverted by an inner linear solve.  A_S p for a block vector p
// (zero outside S) is H^T H p + 2 eta p + lambda V^T Diag(omega(x)) V p +
// 2 kappa VZ^T VZ p + mu p restricted to S: H p on S +- r_z comes from the
// direction pass, XY^T (H p) per slice from the update pass (assign mode),
// and k_majapply adds the z-gather of it to the other terms.
// ---------------------------------------------------------------------------

// Fixed-order sum of count slots (stride doubles apart) from first, the same
// total on every thread of the workgroup: each thread in slot order, the
// wavefronts by DPP moves, then the wavefronts in order.
__device__ __forceinline__ double slots_sum(const double *__restrict__ base, int stride, int first, int count)
{
    __shared__ double red[NT / 64];
    __shared__ double tot;
    double v = 0.0;
    for (int t = threadIdx.x; t < count; t += NT) v += base[(size_t)(first + t) * stride];
    v = wave_sum_last(v);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int w = 0; w < NT / 64; ++w) a += red[w];
        tot = a;
    }
    __syncthreads();
    return tot;
}

template <typename T, int KZ>
__global__ void __launch_bounds__(NT)
k_majapply(Geom g, Params prm, DevState<T> s, const T *__restrict__ qt, const T *__restrict__ x,
           const T *__restrict__ pv, T *__restrict__ ap, const Item *__restrict__ items,
           double *__restrict__ partials)
{
    constexpr int RZ = KZ / 2;
    constexpr int XW = TX + 3, XH = TY + 3;  // x and p at (y0-1+jj, x0-1+ii)
    constexpr int PW = TX + 2, PH = TY + 2;  // w VX p, w VY p at (y0-1+jj, x0-1+ii)
    __shared__ T X[padded<XW, XH>()];
    __shared__ T P[padded<XW, XH>()];
    __shared__ T PX[padded<PW, PH>()];
    __shared__ T PY[padded<PW, PH>()];
    __shared__ double red[NT / 64];

    const Item it = items[blockIdx.z];
    if (s.stop && *s.stop) return;
    const int k = it.k, z0 = it.z0, z1 = it.z0 + it.n;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tx = threadIdx.x & (TX - 1);
    const size_t S = (size_t)g.nx * g.ny;
    Region<XW, XH, 1, 1> rx(g, x0, y0);
#pragma unroll
    for (int qq = 0; qq < rx.E; ++qq) {
        const size_t o = (size_t)k * S + rx.off[qq];
        X[threadIdx.x + qq * NT] = rx.inb[qq] ? x[o] : T(0);
        P[threadIdx.x + qq * NT] = rx.inb[qq] ? pv[o] : T(0);
    }
    // data part at the thread's outputs: sum_c gz_{k+c}[c] qt_{k+c}
    T ht[RPT];
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
        ht[e] = 0;
        const int j = y0 + out_row<RPT>(e), i = x0 + tx;
        if (i >= g.nx || j >= g.ny) continue;
        const size_t o = (size_t)j * g.nx + i;
#pragma unroll
        for (int c = -RZ; c <= RZ; ++c) {
            const int m = k + c;
            if (m < 0 || m >= g.nz) continue;
            ht[e] += s.gz[(size_t)m * KZ + (c + RZ)] * qt[(size_t)m * S + o];
        }
    }
    __syncthreads();
    // omega from x, omega VX p and omega VY p; zero outside the slice
    const T del2 = (T)(prm.delta * prm.delta);
    {
        constexpr int N = PW * PH, E = cdiv(N, NT);
#pragma unroll
        for (int qq = 0; qq < E; ++qq) {
            const int e = threadIdx.x + qq * NT;
            if (e < N) {
                const int jj = e / PW, ii = e - jj * PW;
                const int j = y0 - 1 + jj, i = x0 - 1 + ii;
                T px = 0, py = 0;
                if (i >= 0 && i < g.nx && j >= 0 && j < g.ny) {
                    const T *xc = X + jj * XW + ii;
                    const T *pc = P + jj * XW + ii;
                    const bool hx = i < g.nx - 1, hy = j < g.ny - 1;
                    const T dxv = hx ? xc[1] - xc[0] : T(0), dyv = hy ? xc[XW] - xc[0] : T(0);
                    const T w = inv_sqrt(dxv * dxv + dyv * dyv + del2);
                    px = w * (hx ? pc[1] - pc[0] : T(0));
                    py = w * (hy ? pc[XW] - pc[0] : T(0));
                }
                PX[e] = px;
                PY[e] = py;
            }
        }
    }
    __syncthreads();
    const T lam = (T)prm.lambda, eta2 = (T)(2.0 * prm.eta), kap2 = (T)(2.0 * prm.kappa), mu = (T)prm.mu;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
        const int lj = out_row<RPT>(e), li = tx;
        const int j = y0 + lj, i = x0 + li;
        if (i >= g.nx || j >= g.ny) continue;
        const int pc = (lj + 1) * PW + (li + 1);
        const T tv = PX[pc - 1] - PX[pc] + PY[pc - PW] - PY[pc];
        const T pval = P[(lj + 1) * XW + (li + 1)];
        T a = ht[e] + eta2 * pval;
        a += lam * tv;
        const size_t o = (size_t)k * S + (size_t)j * g.nx + i;
        if (prm.kappa != 0.0) {
            // VZ^T VZ p with p zero outside the block
            const T pm = (k - 1 >= z0) ? pv[o - S] : T(0), pp = (k + 1 < z1) ? pv[o + S] : T(0);
            T zz = 0;
            if (k >= 1) zz += pval - pm;
            if (k < g.nz - 1) zz -= pp - pval;
            a += kap2 * zz;
        }
        a += mu * pval;
        ap[o] = a;
        acc += (double)pval * (double)a;
    }
    double q1[1] = {acc};
    wg_reduce_store<1>(q1, red, partials + slot_of(vb_native()));
}

// Elementwise stages of the inner solve on the gradient items of a launch
// group (tile TX x TY, four outputs a thread); the first workgroup of a block
// (its first slice, tile 0) keeps the block's scalars.  Scalars that a stage
// reads are written by another stage (rho and done are double-buffered by
// iteration parity), so no launch reads what it writes.
template <typename T>
__global__ void __launch_bounds__(NT)
k_cg(int stage, Geom g, DevState<T> s, const Item *__restrict__ items, CgBufs<T> b, int parity, double tol_inner)
{
    const Item it = items[blockIdx.z];
    if (s.stop && *s.stop) return;
    const int k = it.k, blk = it.block;
    const int ntiles = gridDim.x * gridDim.y;
    const bool first = (k == it.z0) && blockIdx.x == 0 && blockIdx.y == 0;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tx = threadIdx.x & (TX - 1);
    const size_t S = (size_t)g.nx * g.ny;
    double *cs = b.cgs + (size_t)CG_STRIDE * blk;
    size_t o[RPT];
    bool in[RPT];
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
        const int j = y0 + out_row<RPT>(e), i = x0 + tx;
        in[e] = i < g.nx && j < g.ny;
        o[e] = in[e] ? (size_t)k * S + (size_t)j * g.nx + i : 0;
    }
    if (stage == CG_INIT) {
        // r = b - A v = -g with v = 0, p = r
#pragma unroll
        for (int e = 0; e < RPT; ++e)
            if (in[e]) {
                const T r = -s.g[o[e]];
                b.r[o[e]] = r;
                b.p[o[e]] = r;
                b.v[o[e]] = 0;
            }
        if (first) {
            const double gg = slots_sum(b.pg, NQG, it.h0 * ntiles, it.hn * ntiles);
            if (threadIdx.x == 0) {
                cs[0] = cs[1] = gg;  // rho = <r, r>
                cs[2] = cs[3] = 0.0;  // not done
                cs[4] = sqrt(gg);     // ||r_0||
                cs[5] = 0.0;          // iterations
                cs[6] = gg;           // ||r||^2 at the end
                cs[7] = gg;           // ||g||^2
            }
        }
        return;
    }
    if (stage == CG_FINAL) {
        // the direction and update passes then apply d' = v (as -g, u = (1, 0))
#pragma unroll
        for (int e = 0; e < RPT; ++e)
            if (in[e]) s.g[o[e]] = -b.v[o[e]];
        if (first && threadIdx.x == 0) {
            double *inf = b.info + 8 * (size_t)blk;
            inf[0] = cs[5];
            inf[1] = cs[6];
            inf[2] = 0.0;
            inf[3] = -cs[7];
            inf[4] = inf[5] = inf[6] = 0.0;
            inf[7] = cs[7];
        }
        return;
    }
    const double rho = cs[parity];
    const bool done = cs[2 + parity] != 0.0;
    const double den = slots_sum(b.pa, 1, it.h0 * ntiles, it.hn * ntiles);
    const bool active = !done && rho != 0.0 && den != 0.0;
    if (stage == CG_VEC) {
        // v += alpha p, r -= alpha A p, alpha = <r, r> / <p, A p>; then <r, r>
        const T alpha = active ? (T)(rho / den) : T(0);
        double rr = 0.0;
#pragma unroll
        for (int e = 0; e < RPT; ++e)
            if (in[e]) {
                T r = b.r[o[e]];
                if (active) {
                    b.v[o[e]] += alpha * b.p[o[e]];
                    r -= alpha * b.ap[o[e]];
                    b.r[o[e]] = r;
                }
                rr += (double)r * (double)r;
            }
        __shared__ double red[NT / 64];
        double q1[1] = {rr};
        wg_reduce_store<1>(q1, red, b.prr + slot_of(vb_native()));
        return;
    }
    // CG_DIR: stop at the tolerance, else p = r + beta p, beta = <r, r>_new / <r, r>
    const double rr = slots_sum(b.prr, 1, it.h0 * ntiles, it.hn * ntiles);
    const bool stop = !active || (tol_inner > 0.0 && sqrt(rr) <= tol_inner * cs[4]);
    if (!stop) {
        const T beta = (T)(rr / rho);
#pragma unroll
        for (int e = 0; e < RPT; ++e)
            if (in[e]) b.p[o[e]] = b.r[o[e]] + beta * b.p[o[e]];
    }
    if (first && threadIdx.x == 0) {
        cs[2 + (parity ^ 1)] = (done || stop) ? 1.0 : 0.0;
        cs[parity ^ 1] = rr;
        if (active) {
            cs[5] += 1.0;
            cs[6] = rr;
        }
    }
}

// ---------------------------------------------------------------------------
// Fused batch passes: one launch runs a pass of the same colour index for
// every problem of a batch, each problem's workgroups a contiguous part of
// the grid (work lists concatenated; each problem gets as many workgroups as
// its own launch would have).  The bodies are the single-problem passes', so
// a fused run is bitwise a run of the problems one by one.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool fused_part(const FusedArgs<T> *__restrict__ fa, const unsigned char *__restrict__ owner,
                                           int *p, VB *vb)
{
    // uniform over the workgroup: the argument block is read with scalar loads
    *p = __builtin_amdgcn_readfirstlane((int)owner[blockIdx.x >> 3]);
    const FusedArgs<T> &a = fa[*p];
    const unsigned l = blockIdx.x - a.wg0, per = a.gx * a.gy;
    if (l >= per * (unsigned)a.nitems) return false;  // padding to the next multiple of 8
    // the divisions run on the vector unit: their (uniform) results are moved
    // back to scalar registers, as the hardware block index would be
    const unsigned bx = l % a.gx, by = (l / a.gx) % a.gy, bz = l / per;
    *vb = VB{(unsigned)__builtin_amdgcn_readfirstlane((int)bx), (unsigned)__builtin_amdgcn_readfirstlane((int)by),
             (unsigned)__builtin_amdgcn_readfirstlane((int)bz), a.gx, a.gy, (unsigned)a.nitems};
    return true;
}

template <typename T, int KZ>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 4)))
k_grad_fused(const FusedArgs<T> *__restrict__ fa, const unsigned char *__restrict__ owner)
{
    int p;
    VB vb;
    if (!fused_part(fa, owner, &p, &vb)) return;
    const FusedArgs<T> &a = fa[p];
    grad_body<T, KZ, false, true>(vb, a.g, a.prm, a.s, a.s.q, a.s.x, nullptr, a.items, GM_BLOCK, a.pg, 0);
}

template <typename T, int KZ, int R, int TYK, bool ONE>
__global__ void __launch_bounds__(NT)
k_dirs_fused(const FusedArgs<T> *__restrict__ fa, const unsigned char *__restrict__ owner)
{
    int p;
    VB vb;
    if (!fused_part(fa, owner, &p, &vb)) return;
    const FusedArgs<T> &a = fa[p];
    dirs_body<T, KZ, R, TYK, ONE>(vb, a.g, a.prm, a.s, a.items, a.pd);
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_solve_fused(const FusedArgs<T> *__restrict__ fa, const unsigned char *__restrict__ owner)
{
    int p;
    VB vb;
    if (!fused_part(fa, owner, &p, &vb)) return;
    const FusedArgs<T> &a = fa[p];
    solve_block(a.prm, a.brs[vb.z], a.ntg, a.ntd, a.pg, a.pd, a.u, a.info, a.s.stop);  // a 1 x 1 x blocks grid
}

template <typename T, int R, int TYK>
__global__ void __launch_bounds__(NT)
k_update_fused(const FusedArgs<T> *__restrict__ fa, const unsigned char *__restrict__ owner)
{
    int p;
    VB vb;
    if (!fused_part(fa, owner, &p, &vb)) return;
    const FusedArgs<T> &a = fa[p];
    update_body<T, R, TYK, false>(vb, a.g, a.s, a.items, a.pairs, a.u, 0);
}

// Streaming copy of n 16-byte words, grid-stride over chunks of U NT words:
// each lane issues its U loads (coalesced, NT words apart) before its U
// stores, so U loads per lane are in flight at once.
template <int U>
__global__ void __launch_bounds__(NT) k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                             size_t n)
{
    const size_t stride = (size_t)gridDim.x * NT * U;
    for (size_t base = (size_t)blockIdx.x * NT * U + threadIdx.x; base < n; base += stride) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + (size_t)u * NT;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = base + (size_t)u * NT;
            if (i < n) dst[i] = v[u];
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers: dispatch on the z extent KZ and the in-slice radius R.
// ---------------------------------------------------------------------------
thread_local LaunchEvents g_launch_events;

// A launch of the sweep kernels, timed by its own start and stop events when
// the caller set them (g_launch_events, used by one launch only).
#define BD3MG_LAUNCH(K, GRID, BLOCK, SHM, ST, ...)                                                   \
    do {                                                                                           \
        if (g_launch_events.start) {                                                               \
            const LaunchEvents ev_ = g_launch_events;                                              \
            g_launch_events = LaunchEvents{};                                                      \
            hipExtLaunchKernelGGL(K, GRID, BLOCK, SHM, ST, ev_.start, ev_.stop, 0, __VA_ARGS__);   \
        } else {                                                                                   \
            hipLaunchKernelGGL(K, GRID, BLOCK, SHM, ST, __VA_ARGS__);                              \
        }                                                                                          \
    } while (0)
#define BD3MG_R_SWITCH(r, CALL)                   \
    switch (r) {                                  \
    case 1: { constexpr int R = 1; CALL; } break; \
    case 2: { constexpr int R = 2; CALL; } break; \
    case 3: { constexpr int R = 3; CALL; } break; \
    case 4: { constexpr int R = 4; CALL; } break; \
    default: return hipErrorInvalidValue;         \
    }

#define BD3MG_KZ_SWITCH(kz, CALL)                  \
    switch (kz) {                                  \
    case 1: { constexpr int KZ = 1; CALL; } break; \
    case 3: { constexpr int KZ = 3; CALL; } break; \
    case 5: { constexpr int KZ = 5; CALL; } break; \
    case 7: { constexpr int KZ = 7; CALL; } break; \
    case 9: { constexpr int KZ = 9; CALL; } break; \
    default: return hipErrorInvalidValue;          \
    }

static dim3 grid_of(const Geom &g, int nitems, int ty = TY)
{
    return dim3(g.ntx, (g.ny + ty - 1) / ty, nitems);
}

// Tile heights: 16 or 32 rows in single precision; double precision keeps 16
// (two 32-row double tiles of the direction pass would not fit the LDS budget).
#define BD3MG_TY_SWITCH(ty, CALL)                                  \
    if constexpr (sizeof(T) == 8) {                                \
        if (ty != 16) return hipErrorInvalidValue;                 \
        constexpr int TYK = 16;                                    \
        CALL;                                                      \
    } else {                                                       \
        switch (ty) {                                              \
        case 16: { constexpr int TYK = 16; CALL; } break;          \
        case 32: { constexpr int TYK = 32; CALL; } break;          \
        default: return hipErrorInvalidValue;                      \
        }                                                          \
    }

template <typename T>
hipError_t launch_grad(const Geom &g, const Params &prm, const DevState<T> &s, const T *q, const T *x,
                       T *out, const Item *items, int nitems, int mode, double *partials, hipStream_t st,
                       int nshare)
{
    if (nitems <= 0) return hipSuccess;
    if (nshare > 0 && g.rz != 0) return hipErrorInvalidValue;
#define BD3MG_GRAD_LAUNCH(TV, BL, STR)                                                             \
    BD3MG_KZ_SWITCH(2 * g.rz + 1, BD3MG_LAUNCH((k_grad<T, KZ, TV, BL, STR>), grid_of(g, nitems), dim3(NT), 0, \
                                               st, g, prm, s, q, x, out, items, mode, partials, nshare))
    const bool blk = mode == GM_BLOCK;
    if (prm.tv3d) {
        if (blk) {
            BD3MG_GRAD_LAUNCH(true, true, false);
        } else {
            BD3MG_GRAD_LAUNCH(true, false, false);
        }
    } else {
        if (blk && s.nt) {
            BD3MG_GRAD_LAUNCH(false, true, true);
        } else if (blk) {
            BD3MG_GRAD_LAUNCH(false, true, false);
        } else {
            BD3MG_GRAD_LAUNCH(false, false, false);
        }
    }
#undef BD3MG_GRAD_LAUNCH
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dirs(const Geom &g, const Params &prm, const DevState<T> &s, const Item *units,
                       int nunits, double *partials, hipStream_t st, bool one)
{
    if (nunits <= 0) return hipSuccess;
    if (one) {
        BD3MG_KZ_SWITCH(2 * g.rz + 1, BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_dirs,
                        BD3MG_LAUNCH((k_dirs<T, KZ, R, TYK, true>), grid_of(g, nunits, TYK), dim3(NT), 0,
                                           st, g, prm, s, units, partials))));
    } else {
        BD3MG_KZ_SWITCH(2 * g.rz + 1, BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_dirs,
                        BD3MG_LAUNCH((k_dirs<T, KZ, R, TYK, false>), grid_of(g, nunits, TYK), dim3(NT), 0,
                                           st, g, prm, s, units, partials))));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const Geom &g, const DevState<T> &s, const Item *items, int nitems,
                         const int2 *pairs, const double *u, bool multi, hipStream_t st, int assign)
{
    if (nitems <= 0) return hipSuccess;
    if (multi) {
        BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_update,
                       BD3MG_LAUNCH((k_update<T, R, TYK, true, false>), grid_of(g, nitems, TYK), dim3(NT), 0,
                                          st, g, s, items, pairs, u, assign)));
    } else if (s.nt) {
        BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_update,
                       BD3MG_LAUNCH((k_update<T, R, TYK, false, true>), grid_of(g, nitems, TYK), dim3(NT), 0,
                                          st, g, s, items, pairs, u, assign)));
    } else {
        BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_update,
                       BD3MG_LAUNCH((k_update<T, R, TYK, false, false>), grid_of(g, nitems, TYK), dim3(NT), 0,
                                          st, g, s, items, pairs, u, assign)));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fused(int pass, const Geom &g, const FusedArgs<T> *fa, const unsigned char *owner, unsigned nwg,
                        hipStream_t st, bool one)
{
    if (nwg == 0) return hipSuccess;
    const dim3 grid(nwg);
    switch (pass) {
    case FP_GRAD:
        BD3MG_KZ_SWITCH(2 * g.rz + 1, BD3MG_LAUNCH((k_grad_fused<T, KZ>), grid, dim3(NT), 0, st, fa, owner));
        break;
    case FP_DIRS:
        if (one) {
            BD3MG_KZ_SWITCH(2 * g.rz + 1, BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_dirs,
                            BD3MG_LAUNCH((k_dirs_fused<T, KZ, R, TYK, true>), grid, dim3(NT), 0, st, fa, owner))));
        } else {
            BD3MG_KZ_SWITCH(2 * g.rz + 1, BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_dirs,
                            BD3MG_LAUNCH((k_dirs_fused<T, KZ, R, TYK, false>), grid, dim3(NT), 0, st, fa, owner))));
        }
        break;
    case FP_SOLVE:
        BD3MG_LAUNCH((k_solve_fused<T>), grid, dim3(NT), 0, st, fa, owner);
        break;
    case FP_UPDATE:
        BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_update,
                       BD3MG_LAUNCH((k_update_fused<T, R, TYK>), grid, dim3(NT), 0, st, fa, owner)));
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_majapply(const Geom &g, const Params &prm, const DevState<T> &s, const T *qt, const T *x,
                           const T *pv, T *ap, const Item *items, int nitems, double *partials, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    BD3MG_KZ_SWITCH(2 * g.rz + 1,
                    BD3MG_LAUNCH((k_majapply<T, KZ>), grid_of(g, nitems), dim3(NT), 0, st, g, prm, s, qt, x,
                                 pv, ap, items, partials));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg(int stage, const Geom &g, const DevState<T> &s, const Item *items, int nitems,
                     const CgBufs<T> &b, int parity, double tol_inner, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    BD3MG_LAUNCH((k_cg<T>), grid_of(g, nitems), dim3(NT), 0, st, stage, g, s, items, b, parity, tol_inner);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_refresh(const Geom &g, const DevState<T> &s, const T *src, T *qout, const Item *items,
                          int nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    BD3MG_KZ_SWITCH(2 * g.rz + 1, BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_aux,
                    BD3MG_LAUNCH((k_refresh<T, KZ, R, TYK>), grid_of(g, nitems, TYK), dim3(NT), 0,
                                       st, g, s, src, qout, items))));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_H(const Geom &g, const DevState<T> &s, const T *in, const T *sub, T *out,
                    const Item *items, int nitems, double *partials, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    BD3MG_KZ_SWITCH(2 * g.rz + 1, BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_aux,
                    BD3MG_LAUNCH((k_H<T, KZ, R, TYK>), grid_of(g, nitems, TYK), dim3(NT), 0, st,
                                       g, s, in, sub, out, items, partials))));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_blurT(const Geom &g, const DevState<T> &s, const T *in, T *out, const Item *items,
                        int nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    BD3MG_R_SWITCH(g.R, BD3MG_TY_SWITCH(g.ty_aux,
                   BD3MG_LAUNCH((k_blurT<T, R, TYK>), grid_of(g, nitems, TYK), dim3(NT), 0, st,
                                      g, s, in, out, items)));
    return hipGetLastError();
}

hipError_t launch_solve(const Params &prm, const BlockRange *br, int nbr, int ntiles_g, int ntiles_d,
                        const double *pg, const double *pd, double *u, double *info, const int *stop,
                        hipStream_t st)
{
    if (nbr <= 0) return hipSuccess;
    BD3MG_LAUNCH(k_solve, dim3(nbr), dim3(NT), 0, st, prm, br, ntiles_g, ntiles_d, pg, pd, u, info,
                       stop);
    return hipGetLastError();
}

hipError_t launch_check(const double *partials, int nslot, double thr, int sweep, int *stop,
                        int *stop_sweep, double *gnorm, hipStream_t st)
{
    hipLaunchKernelGGL(k_check, dim3(1), dim3(NT), 0, st, partials, nslot, thr, sweep, stop, stop_sweep,
                       gnorm);
    return hipGetLastError();
}

hipError_t launch_sum(const double *partials, int nslot, int nq, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(NT), 0, st, partials, nslot, nq, out);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t n16, int variant, hipStream_t st)
{
    const uint4 *a = (const uint4 *)src;
    uint4 *b = (uint4 *)dst;
    switch (variant) {
    case 0:  // one word per lane in flight, 8 workgroups per CU
        hipLaunchKernelGGL(k_copy<1>, dim3(2048), dim3(NT), 0, st, a, b, n16);
        break;
    case 1:  // four words per lane in flight
        hipLaunchKernelGGL(k_copy<4>, dim3(2048), dim3(NT), 0, st, a, b, n16);
        break;
    case 2:  // four words per lane, 32 workgroups per CU
        hipLaunchKernelGGL(k_copy<4>, dim3(8192), dim3(NT), 0, st, a, b, n16);
        break;
    case 3:  // eight words per lane, 16 workgroups per CU
        hipLaunchKernelGGL(k_copy<8>, dim3(4096), dim3(NT), 0, st, a, b, n16);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define BD3MG_RD_SWITCH(r, CALL)                  \
    switch (r) {                                  \
    case 1: { constexpr int R = 1; CALL; } break; \
    case 2: { constexpr int R = 2; CALL; } break; \
    case 3: { constexpr int R = 3; CALL; } break; \
    case 4: { constexpr int R = 4; CALL; } break; \
    case 5: { constexpr int R = 5; CALL; } break; \
    default: return hipErrorInvalidValue;         \
    }

template <typename T>
hipError_t launch_dense(const Geom &g, const Params &prm, const DevState<T> &s, const T *pk, const T *in,
                        const T *sub, T *out, const Item *items, int nitems, int mode, double *partials,
                        hipStream_t st, int nsplit, T *part)
{
    if (nitems <= 0) return hipSuccess;
    if (g.ty_dirs != 16 && g.ty_dirs != 32) return hipErrorInvalidValue;
#define BD3MG_DENSE_TY(CALL)                             \
    if (g.ty_dirs == 16) { constexpr int TYD = 16; CALL; } \
    else { constexpr int TYD = 32; CALL; }
    if (nsplit > 1) {
        // adjoint over source shares into part; the gradient kernel adds them
        if (mode != DM_HT || !part || out) return hipErrorInvalidValue;
        BD3MG_DENSE_TY(
            const dim3 grid(g.ntx, (g.ny + TYD - 1) / TYD, nitems * nsplit);
            BD3MG_RD_SWITCH(g.R, BD3MG_LAUNCH((k_dense<T, R, 1, true, TYD>), grid, dim3(NT), 0, st, g,
                                                    prm, s, pk, in, sub, part, items, mode, nullptr, nsplit)));
        return hipGetLastError();
    }
    BD3MG_DENSE_TY(
        const dim3 grid(g.ntx, (g.ny + TYD - 1) / TYD, nitems);
        if (mode == DM_DIRS) {
            BD3MG_RD_SWITCH(g.R, BD3MG_LAUNCH((k_dense<T, R, 2, false, TYD>), grid, dim3(NT), 0, st, g,
                                                    prm, s, pk, in, sub, out, items, mode, partials, 1));
        } else if (mode == DM_HT) {
            BD3MG_RD_SWITCH(g.R, BD3MG_LAUNCH((k_dense<T, R, 1, true, TYD>), grid, dim3(NT), 0, st, g,
                                                    prm, s, pk, in, sub, out, items, mode, partials, 1));
        } else {
            BD3MG_RD_SWITCH(g.R, BD3MG_LAUNCH((k_dense<T, R, 1, false, TYD>), grid, dim3(NT), 0, st, g,
                                                    prm, s, pk, in, sub, out, items, mode, partials, 1));
        })
#undef BD3MG_DENSE_TY
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_update(const Geom &g, const DevState<T> &s, const Item *items, int nitems,
                               const int2 *pairs, const double *u, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const size_t S = (size_t)g.nx * g.ny;
    const int gx = (int)std::min<size_t>((S + 4 * NT - 1) / (4 * NT), 1024);
    BD3MG_LAUNCH(k_dense_update<T>, dim3(gx, 1, nitems), dim3(NT), 0, st, g, s, items, pairs, u);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch memory of the entry point that allocates nothing
// (bd3mg_run_noalloc): its partial sums, per-block coefficients, stop-test
// control block and stored directions H d1, H d2 are carved from this array
// instead of from buffers of the problem.  Each GPU the library runs on holds
// its own copy, at its own address, until the process ends.  In host code the
// array's name is not a device address: only the pointer returned by
// scratch_base is passed to kernels and copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

hipError_t scratch_base(int device, void **ptr)
{
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static void *base[MAXDEV] = {};
    if (device < 0 || device >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!base[device]) {
        // once per device, with that device current
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        base[device] = p;
    }
    *ptr = base[device];
    return hipSuccess;
}

#define BD3MG_INSTANTIATE(T)                                                                      \
    template hipError_t launch_grad<T>(const Geom &, const Params &, const DevState<T> &,          \
                                       const T *, const T *, T *, const Item *, int, int,         \
                                       double *, hipStream_t, int);                               \
    template hipError_t launch_dirs<T>(const Geom &, const Params &, const DevState<T> &,          \
                                       const Item *, int, double *, hipStream_t, bool);           \
    template hipError_t launch_update<T>(const Geom &, const DevState<T> &, const Item *, int,      \
                                         const int2 *, const double *, bool, hipStream_t, int);   \
    template hipError_t launch_majapply<T>(const Geom &, const Params &, const DevState<T> &,      \
                                           const T *, const T *, const T *, T *, const Item *, int, \
                                           double *, hipStream_t);                                \
    template hipError_t launch_cg<T>(int, const Geom &, const DevState<T> &, const Item *, int,    \
                                     const CgBufs<T> &, int, double, hipStream_t);                \
    template hipError_t launch_fused<T>(int, const Geom &, const FusedArgs<T> *,                   \
                                        const unsigned char *, unsigned, hipStream_t, bool);      \
    template hipError_t launch_refresh<T>(const Geom &, const DevState<T> &, const T *, T *,       \
                                          const Item *, int, hipStream_t);                        \
    template hipError_t launch_H<T>(const Geom &, const DevState<T> &, const T *, const T *, T *,  \
                                    const Item *, int, double *, hipStream_t);                    \
    template hipError_t launch_blurT<T>(const Geom &, const DevState<T> &, const T *, T *,         \
                                        const Item *, int, hipStream_t);

#define BD3MG_INSTANTIATE_DENSE(T)                                                                \
    template hipError_t launch_dense<T>(const Geom &, const Params &, const DevState<T> &, const T *,  \
                                        const T *, const T *, T *, const Item *, int, int, double *,    \
                                        hipStream_t, int, T *);                                         \
    template hipError_t launch_dense_update<T>(const Geom &, const DevState<T> &, const Item *, int,    \
                                               const int2 *, const double *, hipStream_t);

BD3MG_INSTANTIATE_DENSE(float)
BD3MG_INSTANTIATE_DENSE(double)
BD3MG_INSTANTIATE(float)
BD3MG_INSTANTIATE(double)

}  // namespace bd3mg
