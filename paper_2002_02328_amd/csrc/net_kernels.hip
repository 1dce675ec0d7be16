// gfx950 kernels of the learned warm start x0 = y + net(y): a three-level 3D
// U-Net (3x3x3 convolutions with ReLU, 2x2x2 average pooling, nearest
// upsampling, skip connections by channel stacking, a 1x1x1 head).
//
// The convolutions with 16 or more input channels run on the matrix cores as
// implicit products with bf16 operands and float accumulation
// (v_mfma_f32_16x16x32_bf16):
//   forward and data gradient   D[cout][voxels] = W[cout][(tap, ci)] * X[(tap, ci)][voxels]
//   weight gradient             G[cout][ci]     = g[cout][voxels] * X_tap[voxels][ci]   (per tap)
// Operand layout of one 16x16x32 product for lane l (n = l % 16, q = l / 16):
// A[row n][k = 8q .. 8q + 7], B[k = 8q .. 8q + 7][column n], and the lane
// receives D[rows 4q .. 4q + 3][column n].
#include "net_internal.h"

namespace bd3net {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ inline uint32_t bf_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ inline float bf_val(uint32_t b) { return __uint_as_float(b << 16); }
__device__ inline float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ inline uint32_t pack2(float lo, float hi) { return bf_bits(lo) | (bf_bits(hi) << 16); }
// bf16 value > 0 (sign clear, not zero)
__device__ inline bool pos_lo(uint32_t w) { return (w & 0x8000u) == 0 && (w & 0x7fffu) != 0; }
__device__ inline bool pos_hi(uint32_t w) { return (w & 0x80000000u) == 0 && (w & 0x7fff0000u) != 0; }

__device__ inline bf16x8 as_bf8(u32x4 u) { return __builtin_bit_cast(bf16x8, u); }

struct Tile {
    int b, z0, y0, x0;
};

__device__ inline Tile tile_of(int t, int ntx, int nty, int ntz, int tz = CTZ)
{
    Tile r;
    r.x0 = (t % ntx) * CTX;
    t /= ntx;
    r.y0 = (t % nty) * CTY;
    t /= nty;
    r.z0 = (t % ntz) * tz;
    r.b = t / ntz;
    return r;
}

__device__ inline size_t vox_of(const Vol &v, int b, int z, int y, int x)
{
    return (((size_t)b * v.D + z) * v.H + y) * v.W + x;
}

// Eight channels [c, c + 8) of the layer input at voxel (z, y, x) of the output grid.
template <int CIN, int SRC>
__device__ inline u32x4 load_unit(const ConvIn &in, const Vol &v, int b, int z, int y, int x, int c)
{
    if constexpr (SRC == SRC_PLAIN) {
        return *(const u32x4 *)(in.a + vox_of(v, b, z, y, x) * CIN + c);
    } else if constexpr (SRC == SRC_UP) {
        const Vol h = v.half();
        return *(const u32x4 *)(in.a + vox_of(h, b, z >> 1, y >> 1, x >> 1) * CIN + c);
    } else {
        const size_t vx = vox_of(v, b, z, y, x);
        if (c < in.ca) return *(const u32x4 *)(in.a + vx * in.ca + c);
        return *(const u32x4 *)(in.b + vx * (CIN - in.ca) + (c - in.ca));
    }
}

struct ConvArgs {
    Vol v;
    ConvIn in;
    const bf16_t *w;
    const float *bias;
    int split;
    const bf16_t *mask;
    bf16_t *out_b;
    float *out_f;
    int ntx, nty, ntz;
};

// One workgroup: a TZ x CTY x CTX output tile, every output channel, with
// 128 TZ threads.  The input tile with its one-voxel halo is staged in LDS, 32
// channels at a time (16 when the layer has 16), with a 16-byte pad per voxel
// so that the 16 voxels of a matrix column fall on distinct banks.  Wave w
// owns tile rows 4w .. 4w + 3 (a row is 16 voxels along x, one matrix column
// block).  Deeper tiles re-read less halo per output.
template <int CIN, int COUT, int SRC, int MODE, int TZ>
__global__ void __launch_bounds__(128 * TZ) k_conv(ConvArgs a)
{
    constexpr int NTHR = 128 * TZ;
    constexpr int CC = CIN < 32 ? CIN : 32;
    constexpr int NCH = CIN / CC;
    constexpr int PE = CC + 8;
    constexpr int HY = CTY + 2, HX = CTX + 2;
    constexpr int NHV = (TZ + 2) * HY * HX;
    constexpr int UPV = CC / 8;
    constexpr int NKS = (27 * CC + 31) / 32;
    constexpr int MT = COUT / 16;
    constexpr int KP = (27 * CIN + 31) / 32 * 32;
    static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channel counts");
    __shared__ __attribute__((aligned(16))) bf16_t lds[NHV * PE];

    const Tile T = tile_of(blockIdx.x, a.ntx, a.nty, a.ntz, TZ);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;

    f32x4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mt][r] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int ch = 0; ch < NCH; ++ch) {
        if (ch) __syncthreads();
        for (int u = threadIdx.x; u < NHV * UPV; u += NTHR) {
            const int hv = u / UPV, part = u - hv * UPV;
            const int hz = hv / (HY * HX), rem = hv - hz * (HY * HX);
            const int hy = rem / HX, hx = rem - hy * HX;
            const int z = T.z0 + hz - 1, y = T.y0 + hy - 1, x = T.x0 + hx - 1;
            u32x4 val = u32x4{0u, 0u, 0u, 0u};
            if (z >= 0 && z < a.v.D && y >= 0 && y < a.v.H && x >= 0 && x < a.v.W)
                val = load_unit<CIN, SRC>(a.in, a.v, T.b, z, y, x, ch * CC + part * 8);
            *(u32x4 *)(lds + hv * PE + part * 8) = val;
        }
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < NKS; ++ks) {
            const int kk = ks * 32 + 8 * q;
            const int tap = kk / CC, ci = kk - tap * CC;
            const int tv = tap < 27 ? tap : 26;  // padded taps have zero weights
            const int dz = tv / 9, dy = (tv / 3) % 3, dx = tv % 3;
            const int kg = tap * CIN + ch * CC + ci;
            bf16x8 A[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                A[mt] = as_bf8(*(const u32x4 *)(a.w + (size_t)(mt * 16 + n) * KP + kg));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wave * 4 + r;
                const int zr = row / CTY, yr = row - zr * CTY;
                const int hv = ((zr + dz) * HY + (yr + dy)) * HX + n + dx;
                const bf16x8 B = as_bf8(*(const u32x4 *)(lds + hv * PE + ci));
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B, acc[mt][r], 0, 0, 0);
            }
        }
    }

#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = wave * 4 + r;
        const int z = T.z0 + row / CTY, y = T.y0 + row % CTY, x = T.x0 + n;
        if (z >= a.v.D || y >= a.v.H || x >= a.v.W) continue;
        const size_t vx = vox_of(a.v, T.b, z, y, x);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int co = mt * 16 + 4 * q;
            const f32x4 s = acc[mt][r];
            if constexpr (MODE == 0) {
                const float v0 = fmaxf(s[0] + a.bias[co], 0.f), v1 = fmaxf(s[1] + a.bias[co + 1], 0.f);
                const float v2 = fmaxf(s[2] + a.bias[co + 2], 0.f), v3 = fmaxf(s[3] + a.bias[co + 3], 0.f);
                *(u32x2 *)(a.out_b + vx * COUT + co) = u32x2{pack2(v0, v1), pack2(v2, v3)};
            } else {
                if (co < a.split) {
                    const u32x2 m = *(const u32x2 *)(a.mask + vx * a.split + co);
                    const float v0 = pos_lo(m[0]) ? s[0] : 0.f, v1 = pos_hi(m[0]) ? s[1] : 0.f;
                    const float v2 = pos_lo(m[1]) ? s[2] : 0.f, v3 = pos_hi(m[1]) ? s[3] : 0.f;
                    *(u32x2 *)(a.out_b + vx * a.split + co) = u32x2{pack2(v0, v1), pack2(v2, v3)};
                } else {
                    *(f32x4 *)(a.out_f + vx * (COUT - a.split) + (co - a.split)) = s;
                }
            }
        }
    }
}

struct WgArgs {
    Vol v;
    const bf16_t *g;
    ConvIn in;
    float *part, *partb;
    int ntx, nty, ntz, ntiles;
};

// Weight gradient.  Each workgroup sums over a fixed set of tiles (tile t goes
// to workgroup t mod grid), 16 input channels at a time.  Per tile, g (cout
// channels) and the haloed input are staged in LDS channel-major, so the
// eight consecutive voxels of a k-group are contiguous.  The contraction
// index is the tile-linear voxel v = 32 ks + 8 q + i (rows of 16 along x);
// nine wavefronts, wave w owning the three taps (dz, dy) = (w / 3, w % 3),
// dx = 0, 1, 2: the input row is read once from a 16-byte aligned base and
// shifted by dx elements in registers for each of the three taps.
constexpr int WG_THREADS = 9 * 64;

template <int CIN, int COUT, int SRC>
__global__ void __launch_bounds__(WG_THREADS) k_wgrad(WgArgs a)
{
    constexpr int MT = COUT / 16;
    constexpr int NV = CTZ * CTY * CTX;  // 256
    constexpr int GP = NV + 8;
    constexpr int HY = CTY + 2, HXP = 24;  // halo x extent 18, padded to 24
    constexpr int IP = (CTZ + 2) * HY * HXP + 8;
    constexpr int NCH = CIN / 16;
    constexpr int GU = COUT / 8;
    static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channel counts");
    __shared__ __attribute__((aligned(16))) bf16_t gT[COUT * GP];
    __shared__ __attribute__((aligned(16))) bf16_t inT[16 * IP];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, q = lane >> 4;
    for (int i = tid; i < 16 * IP / 8; i += WG_THREADS) *(u32x4 *)(inT + 8 * i) = u32x4{0u, 0u, 0u, 0u};
    float bsum = 0.f;

    for (int ch = 0; ch < NCH; ++ch) {
        f32x4 acc[3][MT];
#pragma unroll
        for (int ti = 0; ti < 3; ++ti)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[ti][mt] = f32x4{0.f, 0.f, 0.f, 0.f};

        for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
            const Tile T = tile_of(t, a.ntx, a.nty, a.ntz);
            __syncthreads();
            for (int u = tid; u < NV * GU; u += WG_THREADS) {
                const int vl = u / GU, part = u - vl * GU;
                const int zl = vl / (CTY * CTX), yl = (vl / CTX) % CTY, xl = vl % CTX;
                const int z = T.z0 + zl, y = T.y0 + yl, x = T.x0 + xl;
                u32x4 val = u32x4{0u, 0u, 0u, 0u};
                if (z < a.v.D && y < a.v.H && x < a.v.W)
                    val = *(const u32x4 *)(a.g + vox_of(a.v, T.b, z, y, x) * COUT + part * 8);
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    gT[(part * 8 + j) * GP + vl] = (bf16_t)(val[j >> 1] >> (16 * (j & 1)));
            }
            for (int u = tid; u < (CTZ + 2) * HY * (CTX + 2) * 2; u += WG_THREADS) {
                const int hv = u >> 1, part = u & 1;
                const int hz = hv / (HY * (CTX + 2)), rem = hv - hz * (HY * (CTX + 2));
                const int hy = rem / (CTX + 2), hx = rem - hy * (CTX + 2);
                const int z = T.z0 + hz - 1, y = T.y0 + hy - 1, x = T.x0 + hx - 1;
                u32x4 val = u32x4{0u, 0u, 0u, 0u};
                if (z >= 0 && z < a.v.D && y >= 0 && y < a.v.H && x >= 0 && x < a.v.W)
                    val = load_unit<CIN, SRC>(a.in, a.v, T.b, z, y, x, ch * 16 + part * 8);
                const int base = (hz * HY + hy) * HXP + hx;
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    inT[(part * 8 + j) * IP + base] = (bf16_t)(val[j >> 1] >> (16 * (j & 1)));
            }
            __syncthreads();
            if (ch == 0 && tid < COUT) {
                for (int v = 0; v < NV; v += 2) {
                    const uint32_t w = *(const uint32_t *)(gT + tid * GP + v);
                    bsum += bf_lo(w) + bf_hi(w);
                }
            }
#pragma unroll 1
            for (int ks = 0; ks < NV / 32; ++ks) {
                bf16x8 A[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    A[mt] = as_bf8(*(const u32x4 *)(gT + (mt * 16 + n) * GP + ks * 32 + 8 * q));
                const int row = 2 * ks + (q >> 1);
                const int zr = row / CTY, yr = row - zr * CTY, xs = 8 * (q & 1);
                const int dz = wave / 3, dy = wave - 3 * dz;
                const bf16_t *p = inT + n * IP + ((zr + dz) * HY + (yr + dy)) * HXP + xs;
                const u32x4 w0 = *(const u32x4 *)p, w1 = *(const u32x4 *)(p + 8);
                const bf16x8 B[3] = {
                    as_bf8(w0),
                    as_bf8(u32x4{__builtin_amdgcn_alignbyte(w0[1], w0[0], 2),
                                 __builtin_amdgcn_alignbyte(w0[2], w0[1], 2),
                                 __builtin_amdgcn_alignbyte(w0[3], w0[2], 2),
                                 __builtin_amdgcn_alignbyte(w1[0], w0[3], 2)}),
                    as_bf8(u32x4{w0[1], w0[2], w0[3], w1[0]})};
#pragma unroll
                for (int ti = 0; ti < 3; ++ti)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        acc[ti][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B[ti], acc[ti][mt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int ti = 0; ti < 3; ++ti) {
            const int tap = 3 * wave + ti;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int co = mt * 16 + 4 * q + i, ci = ch * 16 + n;
                    a.part[(((size_t)blockIdx.x * COUT + co) * CIN + ci) * 27 + tap] = acc[ti][mt][i];
                }
        }
    }
    if (tid < COUT) a.partb[(size_t)blockIdx.x * COUT + tid] = bsum;
}

// One wavefront per output element: lane l sums partials w = l, l + 64, ...
// in order, then a fixed shuffle tree; the same order on every run.
__global__ void __launch_bounds__(NTH) k_wreduce(const float *__restrict__ part, int nwg, int ne,
                                                 float *__restrict__ out)
{
    const int e = blockIdx.x * (NTH / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (e >= ne) return;
    float s = 0.f;
    for (int w = lane; w < nwg; w += 64) s += part[(size_t)w * ne + e];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) out[e] = s;
}

// First layer (one input channel), one thread per voxel of a CTZ x CTY x CTX
// tile: the haloed input tile is rounded to bf16 once into LDS, then 27 taps
// x 16 outputs per voxel (weights read as uniform scalars).
__global__ void __launch_bounds__(NTH) k_conv0(Vol v, const float *__restrict__ y,
                                               const float *__restrict__ w0,
                                               const float *__restrict__ b0, bf16_t *__restrict__ out,
                                               int ntx, int nty, int ntz)
{
    constexpr int HY = CTY + 2, HX = CTX + 2;
    constexpr int NH = (CTZ + 2) * HY * HX;
    __shared__ float yh[NH];
    const Tile T = tile_of(blockIdx.x, ntx, nty, ntz);
    for (int u = threadIdx.x; u < NH; u += NTH) {
        const int hz = u / (HY * HX), rem = u - hz * (HY * HX), hy = rem / HX, hx = rem - hy * HX;
        const int z = T.z0 + hz - 1, yy = T.y0 + hy - 1, x = T.x0 + hx - 1;
        const bool ok = z >= 0 && z < v.D && yy >= 0 && yy < v.H && x >= 0 && x < v.W;
        yh[u] = ok ? bf_val(bf_bits(y[vox_of(v, T.b, z, yy, x)])) : 0.f;
    }
    __syncthreads();
    const int zl = threadIdx.x / (CTY * CTX), yl = (threadIdx.x / CTX) % CTY, xl = threadIdx.x % CTX;
    const int z = T.z0 + zl, yy = T.y0 + yl, x = T.x0 + xl;
    if (z >= v.D || yy >= v.H || x >= v.W) return;
    float in[27];
#pragma unroll
    for (int tap = 0; tap < 27; ++tap)
        in[tap] = yh[((zl + tap / 9) * HY + yl + (tap / 3) % 3) * HX + xl + tap % 3];
    uint32_t o[8];
#pragma unroll
    for (int c = 0; c < 16; c += 2) {
        float s0 = b0[c], s1 = b0[c + 1];
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            s0 += w0[c * 27 + tap] * in[tap];
            s1 += w0[(c + 1) * 27 + tap] * in[tap];
        }
        o[c / 2] = pack2(fmaxf(s0, 0.f), fmaxf(s1, 0.f));
    }
    const size_t i = vox_of(v, T.b, z, yy, x);
    *(u32x4 *)(out + i * 16) = u32x4{o[0], o[1], o[2], o[3]};
    *(u32x4 *)(out + i * 16 + 8) = u32x4{o[4], o[5], o[6], o[7]};
}

// Weight gradient of the first layer: 432 (output, tap) sums per workgroup,
// two per thread, over the voxels of its tiles (same tile split as k_wgrad).
__global__ void __launch_bounds__(NTH) k_wgrad0(Vol v, const bf16_t *__restrict__ g,
                                                const float *__restrict__ y, float *__restrict__ part,
                                                float *__restrict__ partb, int ntx, int nty, int ntz,
                                                int ntiles)
{
    constexpr int NV = CTZ * CTY * CTX;
    constexpr int HY = CTY + 2, HX = CTX + 2;
    constexpr int NH = (CTZ + 2) * HY * HX;
    __shared__ float yh[NH];
    __shared__ float gs[NV * 17];
    const int tid = threadIdx.x;
    const int p0 = tid, p1 = tid + NTH;
    const int co0 = p0 / 27, t0 = p0 % 27;
    const int co1 = p1 < 432 ? p1 / 27 : 0, t1 = p1 < 432 ? p1 % 27 : 0;
    float s0 = 0.f, s1 = 0.f, bs = 0.f;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile T = tile_of(t, ntx, nty, ntz);
        __syncthreads();
        for (int u = tid; u < NH; u += NTH) {
            const int hz = u / (HY * HX), rem = u - hz * (HY * HX), hy = rem / HX, hx = rem - hy * HX;
            const int z = T.z0 + hz - 1, yy = T.y0 + hy - 1, x = T.x0 + hx - 1;
            const bool ok = z >= 0 && z < v.D && yy >= 0 && yy < v.H && x >= 0 && x < v.W;
            yh[u] = ok ? bf_val(bf_bits(y[vox_of(v, T.b, z, yy, x)])) : 0.f;
        }
        for (int u = tid; u < NV * 8; u += NTH) {
            const int vl = u >> 3, c2 = (u & 7) * 2;
            const int zl = vl / (CTY * CTX), yl = (vl / CTX) % CTY, xl = vl % CTX;
            const int z = T.z0 + zl, yy = T.y0 + yl, x = T.x0 + xl;
            uint32_t w = 0;
            if (z < v.D && yy < v.H && x < v.W) w = *(const uint32_t *)(g + vox_of(v, T.b, z, yy, x) * 16 + c2);
            gs[vl * 17 + c2] = bf_lo(w);
            gs[vl * 17 + c2 + 1] = bf_hi(w);
        }
        __syncthreads();
        const int dz0 = t0 / 9, dy0 = (t0 / 3) % 3, dx0 = t0 % 3;
        const int dz1 = t1 / 9, dy1 = (t1 / 3) % 3, dx1 = t1 % 3;
        for (int vl = 0; vl < NV; ++vl) {
            const int zl = vl / (CTY * CTX), yl = (vl / CTX) % CTY, xl = vl % CTX;
            s0 += gs[vl * 17 + co0] * yh[((zl + dz0) * HY + yl + dy0) * HX + xl + dx0];
            s1 += gs[vl * 17 + co1] * yh[((zl + dz1) * HY + yl + dy1) * HX + xl + dx1];
        }
        if (tid < 16)
            for (int vl = 0; vl < NV; ++vl) bs += gs[vl * 17 + tid];
    }
    part[((size_t)blockIdx.x * 16 + co0) * 27 + t0] = s0;
    if (p1 < 432) part[((size_t)blockIdx.x * 16 + co1) * 27 + t1] = s1;
    if (tid < 16) partb[(size_t)blockIdx.x * 16 + tid] = bs;
}

__global__ void __launch_bounds__(NTH) k_head_fwd(Vol v, const bf16_t *__restrict__ e1,
                                                  const float *__restrict__ y, const float *__restrict__ wh,
                                                  const float *__restrict__ bh, float *__restrict__ x0)
{
    const size_t i = (size_t)blockIdx.x * NTH + threadIdx.x;
    if (i >= v.voxels()) return;
    const u32x4 a = *(const u32x4 *)(e1 + i * 16), b = *(const u32x4 *)(e1 + i * 16 + 8);
    float s = bh[0];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        s += wh[2 * j] * bf_lo(a[j]) + wh[2 * j + 1] * bf_hi(a[j]);
        s += wh[8 + 2 * j] * bf_lo(b[j]) + wh[9 + 2 * j] * bf_hi(b[j]);
    }
    x0[i] = y[i] + s;
}

constexpr int NHP = 18;  // head partials: 16 weight sums, bias sum, squared error

__global__ void __launch_bounds__(NTH) k_head_bwd(Vol v, const bf16_t *__restrict__ e1,
                                                  const float *__restrict__ x0, const float *__restrict__ tg,
                                                  const float *__restrict__ wh, bf16_t *__restrict__ g9,
                                                  double *__restrict__ part, float two_over_n)
{
    __shared__ double red[NHP][NTH];
    const size_t i = (size_t)blockIdx.x * NTH + threadIdx.x;
    const int tid = threadIdx.x;
    double loc[NHP];
#pragma unroll
    for (int j = 0; j < NHP; ++j) loc[j] = 0.0;
    if (i < v.voxels()) {
        const float d = x0[i] - tg[i];
        const float gh = two_over_n * d;
        const u32x4 a = *(const u32x4 *)(e1 + i * 16), b = *(const u32x4 *)(e1 + i * 16 + 8);
        float e[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            e[2 * j] = bf_lo(a[j]);
            e[2 * j + 1] = bf_hi(a[j]);
            e[8 + 2 * j] = bf_lo(b[j]);
            e[9 + 2 * j] = bf_hi(b[j]);
        }
        uint32_t o[8];
#pragma unroll
        for (int c = 0; c < 16; c += 2) {
            const float g0 = e[c] > 0.f ? gh * wh[c] : 0.f;
            const float g1 = e[c + 1] > 0.f ? gh * wh[c + 1] : 0.f;
            o[c / 2] = pack2(g0, g1);
        }
        *(u32x4 *)(g9 + i * 16) = u32x4{o[0], o[1], o[2], o[3]};
        *(u32x4 *)(g9 + i * 16 + 8) = u32x4{o[4], o[5], o[6], o[7]};
#pragma unroll
        for (int c = 0; c < 16; ++c) loc[c] = (double)gh * e[c];
        loc[16] = gh;
        loc[17] = (double)d * d;
    }
#pragma unroll
    for (int j = 0; j < NHP; ++j) red[j][tid] = loc[j];
    __syncthreads();
    for (int s = NTH / 2; s > 0; s >>= 1) {
        if (tid < s)
            for (int j = 0; j < NHP; ++j) red[j][tid] += red[j][tid + s];
        __syncthreads();
    }
    if (tid < NHP) part[(size_t)blockIdx.x * NHP + tid] = red[tid][0];
}

// One wavefront per quantity, as k_wreduce.
__global__ void __launch_bounds__(64) k_head_reduce(const double *__restrict__ part, int nwg,
                                                    float *__restrict__ gw, double *__restrict__ sq)
{
    const int j = blockIdx.x, lane = threadIdx.x;
    double s = 0.0;
    for (int w = lane; w < nwg; w += 64) s += part[(size_t)w * NHP + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) {
        if (j < NHP - 1)
            gw[j] = (float)s;
        else
            *sq = s;
    }
}

// v is the fine grid; one thread per (coarse voxel, 8 channels)
__global__ void __launch_bounds__(NTH) k_pool(Vol v, int c, const bf16_t *__restrict__ s, bf16_t *__restrict__ p)
{
    const Vol h = v.half();
    const int cu = c / 8;
    const size_t i = (size_t)blockIdx.x * NTH + threadIdx.x;
    if (i >= h.voxels() * cu) return;
    const int u = i % cu;
    size_t t = i / cu;
    const size_t vc = t;
    const int x = t % h.W;
    t /= h.W;
    const int y = t % h.H;
    t /= h.H;
    const int z = t % h.D;
    const int b = t / h.D;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 8; ++k) {
        const u32x4 w = *(const u32x4 *)(s + vox_of(v, b, 2 * z + (k >> 2), 2 * y + ((k >> 1) & 1), 2 * x + (k & 1)) * c + 8 * u);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[2 * j] += bf_lo(w[j]);
            acc[2 * j + 1] += bf_hi(w[j]);
        }
    }
    *(u32x4 *)(p + vc * c + 8 * u) =
        u32x4{pack2(acc[0] * 0.125f, acc[1] * 0.125f), pack2(acc[2] * 0.125f, acc[3] * 0.125f),
              pack2(acc[4] * 0.125f, acc[5] * 0.125f), pack2(acc[6] * 0.125f, acc[7] * 0.125f)};
}

// v the fine grid; one thread per (fine voxel, 4 channels)
__global__ void __launch_bounds__(NTH) k_pool_bwd(Vol v, int c, const float *__restrict__ gpart,
                                                  const float *__restrict__ gp, const bf16_t *__restrict__ s,
                                                  bf16_t *__restrict__ gs)
{
    const Vol h = v.half();
    const int cu = c / 4;
    const size_t i = (size_t)blockIdx.x * NTH + threadIdx.x;
    if (i >= v.voxels() * cu) return;
    const int u = i % cu;
    size_t t = i / cu;
    const size_t vf = t;
    const int x = t % v.W;
    t /= v.W;
    const int y = t % v.H;
    t /= v.H;
    const int z = t % v.D;
    const int b = t / v.D;
    const f32x4 a = *(const f32x4 *)(gpart + vf * c + 4 * u);
    const f32x4 g = *(const f32x4 *)(gp + vox_of(h, b, z >> 1, y >> 1, x >> 1) * c + 4 * u);
    const u32x2 m = *(const u32x2 *)(s + vf * c + 4 * u);
    const float r0 = pos_lo(m[0]) ? a[0] + 0.125f * g[0] : 0.f;
    const float r1 = pos_hi(m[0]) ? a[1] + 0.125f * g[1] : 0.f;
    const float r2 = pos_lo(m[1]) ? a[2] + 0.125f * g[2] : 0.f;
    const float r3 = pos_hi(m[1]) ? a[3] + 0.125f * g[3] : 0.f;
    *(u32x2 *)(gs + vf * c + 4 * u) = u32x2{pack2(r0, r1), pack2(r2, r3)};
}

// v the fine grid of gu; one thread per (coarse voxel, 4 channels)
__global__ void __launch_bounds__(NTH) k_up_bwd(Vol v, int c, const float *__restrict__ gu,
                                                const bf16_t *__restrict__ e, bf16_t *__restrict__ ge)
{
    const Vol h = v.half();
    const int cu = c / 4;
    const size_t i = (size_t)blockIdx.x * NTH + threadIdx.x;
    if (i >= h.voxels() * cu) return;
    const int u = i % cu;
    size_t t = i / cu;
    const size_t vc = t;
    const int x = t % h.W;
    t /= h.W;
    const int y = t % h.H;
    t /= h.H;
    const int z = t % h.D;
    const int b = t / h.D;
    f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < 8; ++k)
        s += *(const f32x4 *)(gu + vox_of(v, b, 2 * z + (k >> 2), 2 * y + ((k >> 1) & 1), 2 * x + (k & 1)) * c + 4 * u);
    const u32x2 m = *(const u32x2 *)(e + vc * c + 4 * u);
    const float r0 = pos_lo(m[0]) ? s[0] : 0.f, r1 = pos_hi(m[0]) ? s[1] : 0.f;
    const float r2 = pos_lo(m[1]) ? s[2] : 0.f, r3 = pos_hi(m[1]) ? s[3] : 0.f;
    *(u32x2 *)(ge + vc * c + 4 * u) = u32x2{pack2(r0, r1), pack2(r2, r3)};
}

__global__ void __launch_bounds__(NTH) k_pack_fwd(int cin, int cout, int kp, const float *__restrict__ w,
                                                  bf16_t *__restrict__ wk)
{
    const int i = blockIdx.x * NTH + threadIdx.x;
    if (i >= cout * kp) return;
    const int co = i / kp, k = i - co * kp;
    const int tap = k / cin, ci = k - tap * cin;
    wk[i] = tap < 27 ? (bf16_t)bf_bits(w[((size_t)co * cin + ci) * 27 + tap]) : (bf16_t)0;
}

// data gradient weights: wt[ci][k'] with k' = tap' * cout + co, tap' = 26 - tap
__global__ void __launch_bounds__(NTH) k_pack_bwd(int cin, int cout, int kp, const float *__restrict__ w,
                                                  bf16_t *__restrict__ wt)
{
    const int i = blockIdx.x * NTH + threadIdx.x;
    if (i >= cin * kp) return;
    const int ci = i / kp, k = i - ci * kp;
    const int tp = k / cout, co = k - tp * cout;
    wt[i] = tp < 27 ? (bf16_t)bf_bits(w[((size_t)co * cin + ci) * 27 + (26 - tp)]) : (bf16_t)0;
}

__global__ void __launch_bounds__(NTH) k_round(const float *__restrict__ w, float *__restrict__ o, int n)
{
    const int i = blockIdx.x * NTH + threadIdx.x;
    if (i < n) o[i] = bf_val(bf_bits(w[i]));
}

__global__ void __launch_bounds__(NTH) k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, size_t n,
                                              float lr, float b1, float b2, float eps, float bc1, float bc2)
{
    const size_t i = (size_t)blockIdx.x * NTH + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void __launch_bounds__(NTH) k_f64_to_f32(const double *__restrict__ a, float *__restrict__ b, size_t n)
{
    const size_t i = (size_t)blockIdx.x * NTH + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ void __launch_bounds__(NTH) k_f32_to_f64(const float *__restrict__ a, double *__restrict__ b, size_t n)
{
    const size_t i = (size_t)blockIdx.x * NTH + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + NTH - 1) / NTH); }

void tiles(const Vol &v, int &ntx, int &nty, int &ntz, int &ntiles)
{
    ntx = (v.W + CTX - 1) / CTX;
    nty = (v.H + CTY - 1) / CTY;
    ntz = (v.D + CTZ - 1) / CTZ;
    ntiles = ntx * nty * ntz * v.nb;
}

}  // namespace

#define BD3NET_CONV_CASES(X)                                                                      \
    X(16, 16, SRC_PLAIN, 0) X(16, 32, SRC_PLAIN, 0) X(32, 32, SRC_PLAIN, 0) X(32, 64, SRC_PLAIN, 0) \
    X(64, 64, SRC_PLAIN, 0) X(64, 32, SRC_UP, 0) X(64, 32, SRC_CAT, 0) X(32, 16, SRC_UP, 0)       \
    X(32, 16, SRC_CAT, 0) X(16, 32, SRC_PLAIN, 1) X(32, 64, SRC_PLAIN, 1) X(64, 64, SRC_PLAIN, 1) \
    X(64, 32, SRC_PLAIN, 1) X(32, 32, SRC_PLAIN, 1) X(32, 16, SRC_PLAIN, 1) X(16, 16, SRC_PLAIN, 1)

hipError_t conv3(int cin, int cout, int src, int mode, Vol v, ConvIn in, const bf16_t *wk,
                 const float *bias, int split, const bf16_t *mask, bf16_t *out_b, float *out_f,
                 hipStream_t st)
{
    ConvArgs a{v, in, wk, bias, split, mask, out_b, out_f, 0, 0, 0};
    // 4-deep tiles (512 threads, 2.1x halo instead of 2.8x) for the layers
    // with few output channels where they measured faster; 2-deep otherwise
    const int tz = (v.D >= 8 && (cout == 16 || (cin == 32 && cout == 32))) ? 4 : 2;
    a.ntx = (v.W + CTX - 1) / CTX;
    a.nty = (v.H + CTY - 1) / CTY;
    a.ntz = (v.D + tz - 1) / tz;
    const int ntiles = a.ntx * a.nty * a.ntz * v.nb;
    if (ntiles == 0) return hipSuccess;
#define X(CI, CO, S, M)                                                                          \
    if (cin == CI && cout == CO && src == S && mode == M) {                                      \
        if (tz == 4)                                                                             \
            hipLaunchKernelGGL((k_conv<CI, CO, S, M, 4>), dim3(ntiles), dim3(512), 0, st, a);    \
        else                                                                                     \
            hipLaunchKernelGGL((k_conv<CI, CO, S, M, 2>), dim3(ntiles), dim3(256), 0, st, a);    \
        return hipGetLastError();                                                                \
    }
    BD3NET_CONV_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

#define BD3NET_WGRAD_CASES(X)                                                                     \
    X(32, 16, SRC_CAT) X(32, 16, SRC_UP) X(64, 32, SRC_CAT) X(64, 32, SRC_UP) X(64, 64, SRC_PLAIN) \
    X(32, 64, SRC_PLAIN) X(32, 32, SRC_PLAIN) X(16, 32, SRC_PLAIN) X(16, 16, SRC_PLAIN)

hipError_t wgrad3(int cin, int cout, int src, Vol v, const bf16_t *g, ConvIn in, float *part,
                  float *partb, int nwg_max, int *nwg_out, hipStream_t st)
{
    WgArgs a{v, g, in, part, partb, 0, 0, 0, 0};
    tiles(v, a.ntx, a.nty, a.ntz, a.ntiles);
    const int nwg = a.ntiles < nwg_max ? a.ntiles : nwg_max;
    *nwg_out = nwg;
    if (nwg <= 0) return hipErrorInvalidValue;
#define X(CI, CO, S)                                                                           \
    if (cin == CI && cout == CO && src == S) {                                                 \
        hipLaunchKernelGGL((k_wgrad<CI, CO, S>), dim3(nwg), dim3(WG_THREADS), 0, st, a);       \
        return hipGetLastError();                                                              \
    }
    BD3NET_WGRAD_CASES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t wreduce(const float *part, int nwg, int ne, float *out, const float *partb, int nbias,
                   float *outb, hipStream_t st)
{
    constexpr int EPB = NTH / 64;  // elements per block, one wavefront each
    hipLaunchKernelGGL(k_wreduce, dim3((ne + EPB - 1) / EPB), dim3(NTH), 0, st, part, nwg, ne, out);
    hipLaunchKernelGGL(k_wreduce, dim3((nbias + EPB - 1) / EPB), dim3(NTH), 0, st, partb, nwg, nbias, outb);
    return hipGetLastError();
}

hipError_t conv0_fwd(Vol v, const float *y, const float *w0, const float *b0, bf16_t *out, hipStream_t st)
{
    int ntx, nty, ntz, ntiles;
    tiles(v, ntx, nty, ntz, ntiles);
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_conv0, dim3(ntiles), dim3(NTH), 0, st, v, y, w0, b0, out, ntx, nty, ntz);
    return hipGetLastError();
}

hipError_t conv0_wgrad(Vol v, const bf16_t *g, const float *y, float *part, float *partb, int nwg_max,
                       int *nwg_out, hipStream_t st)
{
    int ntx, nty, ntz, ntiles;
    tiles(v, ntx, nty, ntz, ntiles);
    const int nwg = ntiles < nwg_max ? ntiles : nwg_max;
    *nwg_out = nwg;
    if (nwg <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wgrad0, dim3(nwg), dim3(NTH), 0, st, v, g, y, part, partb, ntx, nty, ntz, ntiles);
    return hipGetLastError();
}

hipError_t head_fwd(Vol v, const bf16_t *e1, const float *y, const float *wh, const float *bh, float *x0,
                    hipStream_t st)
{
    if (v.voxels() == 0) return hipSuccess;
    hipLaunchKernelGGL(k_head_fwd, dim3(blocks_for(v.voxels())), dim3(NTH), 0, st, v, e1, y, wh, bh, x0);
    return hipGetLastError();
}

hipError_t head_bwd(Vol v, const bf16_t *e1, const float *x0, const float *t, const float *wh, bf16_t *g9,
                    double *part, int *nwg_out, hipStream_t st)
{
    const unsigned nwg = blocks_for(v.voxels());
    *nwg_out = (int)nwg;
    if (nwg == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_head_bwd, dim3(nwg), dim3(NTH), 0, st, v, e1, x0, t, wh, g9, part,
                       (float)(2.0 / (double)v.voxels()));
    return hipGetLastError();
}

hipError_t head_reduce(const double *part, int nwg, float *gw17, double *sq, hipStream_t st)
{
    hipLaunchKernelGGL(k_head_reduce, dim3(NHP), dim3(64), 0, st, part, nwg, gw17, sq);
    return hipGetLastError();
}

hipError_t pool_fwd(Vol v, int c, const bf16_t *s, bf16_t *p, hipStream_t st)
{
    const size_t n = v.half().voxels() * (c / 8);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pool, dim3(blocks_for(n)), dim3(NTH), 0, st, v, c, s, p);
    return hipGetLastError();
}

hipError_t pool_bwd(Vol v, int c, const float *gpart, const float *gp, const bf16_t *s, bf16_t *gs,
                    hipStream_t st)
{
    const size_t n = v.voxels() * (c / 4);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for(n)), dim3(NTH), 0, st, v, c, gpart, gp, s, gs);
    return hipGetLastError();
}

hipError_t up_bwd(Vol v, int c, const float *gu, const bf16_t *e, bf16_t *ge, hipStream_t st)
{
    const size_t n = v.half().voxels() * (c / 4);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_up_bwd, dim3(blocks_for(n)), dim3(NTH), 0, st, v, c, gu, e, ge);
    return hipGetLastError();
}

hipError_t pack_fwd(int cin, int cout, const float *w, bf16_t *wk, hipStream_t st)
{
    const int kp = kpad(cin);
    hipLaunchKernelGGL(k_pack_fwd, dim3(blocks_for((size_t)cout * kp)), dim3(NTH), 0, st, cin, cout, kp, w, wk);
    return hipGetLastError();
}

hipError_t pack_bwd(int cin, int cout, const float *w, bf16_t *wt, hipStream_t st)
{
    const int kp = kpad(cout);
    hipLaunchKernelGGL(k_pack_bwd, dim3(blocks_for((size_t)cin * kp)), dim3(NTH), 0, st, cin, cout, kp, w, wt);
    return hipGetLastError();
}

hipError_t round_bf16(const float *w, float *out, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_round, dim3(blocks_for(n)), dim3(NTH), 0, st, w, out, n);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                float eps, float bc1, float bc2, hipStream_t st)
{
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(NTH), 0, st, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t f64_to_f32(const double *a, float *b, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_f64_to_f32, dim3(blocks_for(n)), dim3(NTH), 0, st, a, b, n);
    return hipGetLastError();
}

hipError_t f32_to_f64(const float *a, double *b, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks_for(n)), dim3(NTH), 0, st, a, b, n);
    return hipGetLastError();
}

}  // namespace bd3net
