// Internal interface between the host side of the warm-start network
// (net_api.hip) and its gfx950 kernels (net_kernels.hip).  Not part of the ABI.
//
// Activations are bfloat16, channels last: a batch of nb volumes D x H x W with
// C channels is [nb][D][H][W][C].  Gradients that are summed again before
// they feed a matrix product (skip, upsample and pooling paths) are float.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace bd3net {

typedef uint16_t bf16_t;  // bit pattern of a bfloat16

// Output tile of one convolution workgroup and its one-voxel halo.
constexpr int CTZ = 2, CTY = 8, CTX = 16;
constexpr int NTH = 256;

enum Src : int {
    SRC_PLAIN = 0,  // one tensor at the output resolution
    SRC_UP = 1,     // one tensor at half resolution, repeated over 2x2x2 cells
    SRC_CAT = 2     // two tensors at the output resolution, stacked along channels
};

struct Vol {
    int nb, D, H, W;
    __host__ __device__ size_t voxels() const { return (size_t)nb * D * H * W; }
    __host__ __device__ Vol half() const { return Vol{nb, D / 2, H / 2, W / 2}; }
};

// Input of a convolution: a (and b for SRC_CAT, whose first ca channels come
// from a and the rest from b).
struct ConvIn {
    const bf16_t *a;
    const bf16_t *b;
    int ca;
};

// 3x3x3 convolution, zero padding, as a product on the matrix cores.
//  forward (mode 0): y = relu(conv(in; wk) + bias) stored bf16 with cout channels.
//  data gradient (mode 1): acc = conv(g; wt), wt the flipped transpose; output
//    channels below `split` go to out_b (bf16, `split` channels) multiplied by
//    mask > 0, the others to out_f (float, cout - split channels) unmasked.
// wk is [cout][kp] bf16 with k = tap * cin + ci (tap = 9 dz + 3 dy + dx) and kp
// = 27 cin rounded up to 32 (zero padding).
hipError_t conv3(int cin, int cout, int src, int mode, Vol v, ConvIn in, const bf16_t *wk,
                 const float *bias, int split, const bf16_t *mask, bf16_t *out_b, float *out_f,
                 hipStream_t st);

// Weight gradient of a 3x3x3 convolution: part[w][co][ci][tap] and
// partb[w][co] of the nwg workgroups, for the gradient g (cout channels) of the
// pre-activation and the layer input `in` (cin channels).  Returns the number
// of workgroups used in *nwg_out (at most nwg_max).
hipError_t wgrad3(int cin, int cout, int src, Vol v, const bf16_t *g, ConvIn in, float *part,
                  float *partb, int nwg_max, int *nwg_out, hipStream_t st);

// out[e] = sum over w < nwg of part[w * n + e] (fixed order), for both the
// weight partials (n = ne) and the bias partials (n = nb_).
hipError_t wreduce(const float *part, int nwg, int ne, float *out, const float *partb, int nbias,
                   float *outb, hipStream_t st);

// First layer: one float input channel (rounded to bf16), 16 outputs, VALU.
// w0 is [16][27] float (values already bf16), b0 [16].
hipError_t conv0_fwd(Vol v, const float *y, const float *w0, const float *b0, bf16_t *out,
                     hipStream_t st);
hipError_t conv0_wgrad(Vol v, const bf16_t *g, const float *y, float *part, float *partb,
                       int nwg_max, int *nwg_out, hipStream_t st);

// Head: x0 = y + bh + sum_c wh[c] e1[c] (16 channels).
hipError_t head_fwd(Vol v, const bf16_t *e1, const float *y, const float *wh, const float *bh,
                    float *x0, hipStream_t st);
// Mean squared error against t: g9 = (2 (x0 - t) / n) wh[c] [e1 > 0] (bf16),
// partials [w][0 .. 15] = sum gh e1[c], [16] = sum gh, [17] = sum (x0 - t)^2
// (double, fixed order).  n = all voxels of the batch.
hipError_t head_bwd(Vol v, const bf16_t *e1, const float *x0, const float *t, const float *wh,
                    bf16_t *g9, double *part, int *nwg_out, hipStream_t st);
// gw17[0 .. 15] = head weight gradient, gw17[16] = head bias gradient (float),
// *sq = sum of squared errors (double).
hipError_t head_reduce(const double *part, int nwg, float *gw17, double *sq, hipStream_t st);

// 2x2x2 average pooling of c channels (v is the fine grid).
hipError_t pool_fwd(Vol v, int c, const bf16_t *s, bf16_t *p, hipStream_t st);
// g_s = (gpart + gp[cell] / 8) [s > 0] (bf16), v the fine grid.
hipError_t pool_bwd(Vol v, int c, const float *gpart, const float *gp, const bf16_t *s,
                    bf16_t *gs, hipStream_t st);
// g_e = (sum over the cell of gu) [e > 0] (bf16), v the fine grid of gu.
hipError_t up_bwd(Vol v, int c, const float *gu, const bf16_t *e, bf16_t *ge, hipStream_t st);

// Parameters: canonical float layout per layer, weights [cout][cin][27] then bias.
hipError_t pack_fwd(int cin, int cout, const float *w, bf16_t *wk, hipStream_t st);
hipError_t pack_bwd(int cin, int cout, const float *w, bf16_t *wt, hipStream_t st);
hipError_t round_bf16(const float *w, float *out, int n, hipStream_t st);
hipError_t adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1,
                float b2, float eps, float bc1, float bc2, hipStream_t st);

// Precision conversions of whole volumes.
hipError_t f64_to_f32(const double *a, float *b, size_t n, hipStream_t st);
hipError_t f32_to_f64(const float *a, double *b, size_t n, hipStream_t st);

inline int kpad(int cin) { return (27 * cin + 31) / 32 * 32; }

}  // namespace bd3net
