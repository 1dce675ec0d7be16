/*
 * Oracle of the learned warm start: a three-level 3D U-Net mapping an
 * observation y to x0 = y + net(y), trained by mean squared error against
 * BD3MG solutions.  Plain FP64 loops, direct definitions of each layer and of
 * its backward pass.
 *
 * TEST INFRASTRUCTURE ONLY; shares nothing with the HIP implementation.
 *
 * Network (base width c, input channels cin, volumes D x H x W divisible by 4;
 * every conv is 3x3x3 with zero padding and a bias, followed by ReLU unless
 * noted):
 *   a1 = conv(in; cin->c)      s1 = conv(a1; c->c)
 *   p1 = avgpool2(s1)
 *   a2 = conv(p1; c->2c)       s2 = conv(a2; 2c->2c)
 *   p2 = avgpool2(s2)
 *   a3 = conv(p2; 2c->4c)      b3 = conv(a3; 4c->4c)
 *   u2 = up2(b3)               c2 = conv(u2; 4c->2c)
 *   e2 = conv([c2, s2]; 4c->2c)
 *   u1 = up2(e2)               c1 = conv(u1; 2c->c)
 *   e1 = conv([c1, s1]; 2c->c)
 *   h  = conv1x1(e1; c->1), no ReLU
 *   out = in[channel 0] + h
 * avgpool2 averages 2x2x2 cells; up2 repeats each voxel in a 2x2x2 cell;
 * [a, b] stacks channels.
 *
 * Tensors are [C][D][H][W].  Parameters are one flat array, layer by layer in
 * the order above: weights [Cout][Cin][kd][kh][kw] then bias [Cout].
 * With bf16 != 0, the copy of the input fed to the first layer, every stored
 * hidden activation and every weight is rounded to the nearest bfloat16 (ties
 * to even) before use, the storage format of the device implementation; the
 * residual add uses the input as given, biases are not rounded, sums stay in
 * FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NLAYERS 11

typedef struct {
    int cin, cout, k;  /* k = 3 or 1 */
    int relu;
} layer_t;

static void layers_of(int c, int cin0, layer_t *L)
{
    const int spec[NLAYERS][4] = {
        {cin0, c, 3, 1},      {c, c, 3, 1},          {c, 2 * c, 3, 1},     {2 * c, 2 * c, 3, 1},
        {2 * c, 4 * c, 3, 1}, {4 * c, 4 * c, 3, 1},  {4 * c, 2 * c, 3, 1}, {4 * c, 2 * c, 3, 1},
        {2 * c, c, 3, 1},     {2 * c, c, 3, 1},      {c, 1, 1, 0}};
    for (int i = 0; i < NLAYERS; ++i) {
        L[i].cin = spec[i][0];
        L[i].cout = spec[i][1];
        L[i].k = spec[i][2];
        L[i].relu = spec[i][3];
    }
}

static size_t layer_params(const layer_t *l) { return (size_t)l->cout * l->cin * l->k * l->k * l->k + l->cout; }

size_t orcnet_num_params(int c, int cin0)
{
    layer_t L[NLAYERS];
    layers_of(c, cin0, L);
    size_t n = 0;
    for (int i = 0; i < NLAYERS; ++i) n += layer_params(&L[i]);
    return n;
}

/* Round to the nearest bfloat16 (8 significant bits), ties to even. */
double orcnet_round_bf16(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return v; /* inf / nan */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static void round_all(double *a, size_t n, int bf16)
{
    if (!bf16) return;
    for (size_t i = 0; i < n; ++i) a[i] = orcnet_round_bf16(a[i]);
}

/* out[co] = b[co] + sum_ci sum_taps w[co][ci][t] in[ci][v + t - r] (zero padding) */
static void conv_fwd(const layer_t *l, const double *w, const double *b, const double *in, int D, int H,
                     int W, double *out)
{
    const int k = l->k, r = k / 2;
    const size_t V = (size_t)D * H * W;
    for (int co = 0; co < l->cout; ++co)
        for (int z = 0; z < D; ++z)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    double s = b[co];
                    for (int ci = 0; ci < l->cin; ++ci)
                        for (int a = 0; a < k; ++a)
                            for (int bb = 0; bb < k; ++bb)
                                for (int cc = 0; cc < k; ++cc) {
                                    const int zz = z + a - r, yy = y + bb - r, xx = x + cc - r;
                                    if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                                    const double wv = w[(((size_t)co * l->cin + ci) * k + a) * k * k + bb * k + cc];
                                    s += wv * in[(size_t)ci * V + ((size_t)zz * H + yy) * W + xx];
                                }
                    out[(size_t)co * V + ((size_t)z * H + y) * W + x] = s;
                }
}

/* Given g = dL/d(out) (pre-activation), accumulate dL/d(in) into gin (may be
 * NULL), and write dL/dw, dL/db. */
static void conv_bwd(const layer_t *l, const double *w, const double *in, const double *g, int D, int H,
                     int W, double *gin, double *gw, double *gb)
{
    const int k = l->k, r = k / 2;
    const size_t V = (size_t)D * H * W;
    const size_t nw = (size_t)l->cout * l->cin * k * k * k;
    memset(gw, 0, nw * sizeof(double));
    for (int co = 0; co < l->cout; ++co) {
        double sb = 0.0;
        for (size_t v = 0; v < V; ++v) sb += g[(size_t)co * V + v];
        gb[co] = sb;
    }
    for (int co = 0; co < l->cout; ++co)
        for (int z = 0; z < D; ++z)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    const double gv = g[(size_t)co * V + ((size_t)z * H + y) * W + x];
                    if (gv == 0.0) continue;
                    for (int ci = 0; ci < l->cin; ++ci)
                        for (int a = 0; a < k; ++a)
                            for (int bb = 0; bb < k; ++bb)
                                for (int cc = 0; cc < k; ++cc) {
                                    const int zz = z + a - r, yy = y + bb - r, xx = x + cc - r;
                                    if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                                    const size_t wi = (((size_t)co * l->cin + ci) * k + a) * k * k + bb * k + cc;
                                    const size_t ii = (size_t)ci * V + ((size_t)zz * H + yy) * W + xx;
                                    gw[wi] += gv * in[ii];
                                    if (gin) gin[ii] += gv * w[wi];
                                }
                }
}

static void relu(double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (a[i] < 0.0) a[i] = 0.0;
}

/* g *= (a > 0) where a is the post-ReLU activation */
static void relu_bwd(const double *a, double *g, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!(a[i] > 0.0)) g[i] = 0.0;
}

static void pool_fwd(const double *in, int C, int D, int H, int W, double *out)
{
    const int d = D / 2, h = H / 2, w = W / 2;
    for (int c = 0; c < C; ++c)
        for (int z = 0; z < d; ++z)
            for (int y = 0; y < h; ++y)
                for (int x = 0; x < w; ++x) {
                    double s = 0.0;
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b)
                            for (int e = 0; e < 2; ++e)
                                s += in[(((size_t)c * D + 2 * z + a) * H + 2 * y + b) * W + 2 * x + e];
                    out[(((size_t)c * d + z) * h + y) * w + x] = s / 8.0;
                }
}

/* accumulate dL/d(in) += pool^T g */
static void pool_bwd(const double *g, int C, int D, int H, int W, double *gin)
{
    const int d = D / 2, h = H / 2, w = W / 2;
    for (int c = 0; c < C; ++c)
        for (int z = 0; z < D; ++z)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x)
                    gin[(((size_t)c * D + z) * H + y) * W + x] +=
                        g[(((size_t)c * d + z / 2) * h + y / 2) * w + x / 2] / 8.0;
}

/* up2: (C, d, h, w) -> (C, 2d, 2h, 2w) */
static void up_fwd(const double *in, int C, int d, int h, int w, double *out)
{
    const int D = 2 * d, H = 2 * h, W = 2 * w;
    for (int c = 0; c < C; ++c)
        for (int z = 0; z < D; ++z)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x)
                    out[(((size_t)c * D + z) * H + y) * W + x] = in[(((size_t)c * d + z / 2) * h + y / 2) * w + x / 2];
}

/* gin (C, d, h, w) = sum over each 2x2x2 cell of g (C, 2d, 2h, 2w) */
static void up_bwd(const double *g, int C, int d, int h, int w, double *gin)
{
    const int D = 2 * d, H = 2 * h, W = 2 * w;
    for (int c = 0; c < C; ++c)
        for (int z = 0; z < d; ++z)
            for (int y = 0; y < h; ++y)
                for (int x = 0; x < w; ++x) {
                    double s = 0.0;
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b)
                            for (int e = 0; e < 2; ++e)
                                s += g[(((size_t)c * D + 2 * z + a) * H + 2 * y + b) * W + 2 * x + e];
                    gin[(((size_t)c * d + z) * h + y) * w + x] = s;
                }
}

typedef struct {
    layer_t L[NLAYERS];
    const double *w[NLAYERS], *b[NLAYERS];
    double *wr; /* weights as used (rounded copy when bf16) */
} net_t;

static void net_init(net_t *n, int c, int cin0, const double *params, int bf16)
{
    layers_of(c, cin0, n->L);
    size_t tot = orcnet_num_params(c, cin0);
    n->wr = (double *)malloc(tot * sizeof(double));
    memcpy(n->wr, params, tot * sizeof(double));
    size_t off = 0;
    for (int i = 0; i < NLAYERS; ++i) {
        const size_t nw = (size_t)n->L[i].cout * n->L[i].cin * n->L[i].k * n->L[i].k * n->L[i].k;
        round_all(n->wr + off, nw, bf16); /* weights stored in bf16; biases stay FP32-exact */
        n->w[i] = n->wr + off;
        n->b[i] = n->wr + off + nw;
        off += nw + n->L[i].cout;
    }
}

/* Activations of one forward pass. */
typedef struct {
    double *in, *inq, *a1, *s1, *p1, *a2, *s2, *p2, *a3, *b3, *u2, *c2, *cat2, *e2, *u1, *c1, *cat1, *e1, *h;
} acts_t;

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

static void acts_alloc(acts_t *A, int c, int cin0, int D, int H, int W)
{
    const size_t V1 = (size_t)D * H * W, V2 = V1 / 8, V3 = V1 / 64;
    A->in = zalloc(cin0 * V1);
    A->inq = zalloc(cin0 * V1);
    A->a1 = zalloc(c * V1);
    A->s1 = zalloc(c * V1);
    A->p1 = zalloc(c * V2);
    A->a2 = zalloc(2 * c * V2);
    A->s2 = zalloc(2 * c * V2);
    A->p2 = zalloc(2 * c * V3);
    A->a3 = zalloc(4 * c * V3);
    A->b3 = zalloc(4 * c * V3);
    A->u2 = zalloc(4 * c * V2);
    A->c2 = zalloc(2 * c * V2);
    A->cat2 = zalloc(4 * c * V2);
    A->e2 = zalloc(2 * c * V2);
    A->u1 = zalloc(2 * c * V1);
    A->c1 = zalloc(c * V1);
    A->cat1 = zalloc(2 * c * V1);
    A->e1 = zalloc(c * V1);
    A->h = zalloc(V1);
}

static void acts_free(acts_t *A)
{
    double **p = (double **)A;
    for (size_t i = 0; i < sizeof(acts_t) / sizeof(double *); ++i) free(p[i]);
}

static void layer_fwd(const net_t *n, int i, const double *in, int D, int H, int W, double *out, int bf16)
{
    conv_fwd(&n->L[i], n->w[i], n->b[i], in, D, H, W, out);
    const size_t cnt = (size_t)n->L[i].cout * D * H * W;
    if (n->L[i].relu) relu(out, cnt);
    if (n->L[i].relu) round_all(out, cnt, bf16); /* the head's output stays FP32 */
}

static void forward(const net_t *n, acts_t *A, int c, int cin0, int D, int H, int W, int bf16)
{
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4;
    const size_t V1 = (size_t)D * H * W, V2 = V1 / 8;
    /* the first layer sees the input in storage precision; the residual
       x0 = in + h keeps the input as given */
    memcpy(A->inq, A->in, cin0 * V1 * sizeof(double));
    round_all(A->inq, cin0 * V1, bf16);
    layer_fwd(n, 0, A->inq, D, H, W, A->a1, bf16);
    layer_fwd(n, 1, A->a1, D, H, W, A->s1, bf16);
    pool_fwd(A->s1, c, D, H, W, A->p1);
    round_all(A->p1, c * V2, bf16);
    layer_fwd(n, 2, A->p1, D2, H2, W2, A->a2, bf16);
    layer_fwd(n, 3, A->a2, D2, H2, W2, A->s2, bf16);
    pool_fwd(A->s2, 2 * c, D2, H2, W2, A->p2);
    round_all(A->p2, 2 * c * (V2 / 8), bf16);
    layer_fwd(n, 4, A->p2, D3, H3, W3, A->a3, bf16);
    layer_fwd(n, 5, A->a3, D3, H3, W3, A->b3, bf16);
    up_fwd(A->b3, 4 * c, D3, H3, W3, A->u2);
    layer_fwd(n, 6, A->u2, D2, H2, W2, A->c2, bf16);
    memcpy(A->cat2, A->c2, 2 * c * V2 * sizeof(double));
    memcpy(A->cat2 + 2 * c * V2, A->s2, 2 * c * V2 * sizeof(double));
    layer_fwd(n, 7, A->cat2, D2, H2, W2, A->e2, bf16);
    up_fwd(A->e2, 2 * c, D2, H2, W2, A->u1);
    layer_fwd(n, 8, A->u1, D, H, W, A->c1, bf16);
    memcpy(A->cat1, A->c1, c * V1 * sizeof(double));
    memcpy(A->cat1 + c * V1, A->s1, c * V1 * sizeof(double));
    layer_fwd(n, 9, A->cat1, D, H, W, A->e1, bf16);
    layer_fwd(n, 10, A->e1, D, H, W, A->h, bf16);
}

/* out[V] = in[channel 0] + net(in) for one volume of cin0 channels [cin0][D][H][W]. */
void orcnet_forward(int c, int cin0, const double *params, const double *in, int D, int H, int W,
                    int bf16, double *out)
{
    net_t n;
    net_init(&n, c, cin0, params, bf16);
    acts_t A;
    acts_alloc(&A, c, cin0, D, H, W);
    const size_t V1 = (size_t)D * H * W;
    memcpy(A.in, in, cin0 * V1 * sizeof(double));
    forward(&n, &A, c, cin0, D, H, W, bf16);
    for (size_t v = 0; v < V1; ++v) out[v] = A.in[v] + A.h[v];
    acts_free(&A);
    free(n.wr);
}

/* Mean squared error L = (1/V) sum (out - target)^2 over one volume, and dL/dparams
 * (flat, same layout as params).  Returns L. */
double orcnet_loss_grad(int c, int cin0, const double *params, const double *in, const double *target,
                        int D, int H, int W, int bf16, double *grad)
{
    net_t n;
    net_init(&n, c, cin0, params, bf16);
    acts_t A;
    acts_alloc(&A, c, cin0, D, H, W);
    const int D2 = D / 2, H2 = H / 2, W2 = W / 2, D3 = D / 4, H3 = H / 4, W3 = W / 4;
    const size_t V1 = (size_t)D * H * W, V2 = V1 / 8, V3 = V1 / 64;
    memcpy(A.in, in, cin0 * V1 * sizeof(double));
    forward(&n, &A, c, cin0, D, H, W, bf16);
    double loss = 0.0;
    double *gh = zalloc(V1);
    for (size_t v = 0; v < V1; ++v) {
        const double e = A.in[v] + A.h[v] - target[v];
        loss += e * e;
        gh[v] = 2.0 * e / (double)V1;
    }
    loss /= (double)V1;

    double *gw[NLAYERS], *gb[NLAYERS];
    size_t off = 0;
    for (int i = 0; i < NLAYERS; ++i) {
        const size_t nw = (size_t)n.L[i].cout * n.L[i].cin * n.L[i].k * n.L[i].k * n.L[i].k;
        gw[i] = grad + off;
        gb[i] = grad + off + nw;
        off += nw + n.L[i].cout;
    }
    double *ge1 = zalloc(c * V1), *gcat1 = zalloc(2 * c * V1), *gu1 = zalloc(2 * c * V1);
    double *ge2 = zalloc(2 * c * V2), *gcat2 = zalloc(4 * c * V2), *gu2 = zalloc(4 * c * V2);
    double *gb3 = zalloc(4 * c * V3), *ga3 = zalloc(4 * c * V3), *gp2 = zalloc(2 * c * V3);
    double *gs2 = zalloc(2 * c * V2), *ga2 = zalloc(2 * c * V2), *gp1 = zalloc(c * V2);
    double *gs1 = zalloc(c * V1), *ga1 = zalloc(c * V1), *gc1 = zalloc(c * V1), *gc2 = zalloc(2 * c * V2);

    conv_bwd(&n.L[10], n.w[10], A.e1, gh, D, H, W, ge1, gw[10], gb[10]);
    relu_bwd(A.e1, ge1, c * V1);
    conv_bwd(&n.L[9], n.w[9], A.cat1, ge1, D, H, W, gcat1, gw[9], gb[9]);
    memcpy(gc1, gcat1, c * V1 * sizeof(double));
    for (size_t i = 0; i < c * V1; ++i) gs1[i] += gcat1[c * V1 + i];
    relu_bwd(A.c1, gc1, c * V1);
    conv_bwd(&n.L[8], n.w[8], A.u1, gc1, D, H, W, gu1, gw[8], gb[8]);
    up_bwd(gu1, 2 * c, D2, H2, W2, ge2);
    relu_bwd(A.e2, ge2, 2 * c * V2);
    conv_bwd(&n.L[7], n.w[7], A.cat2, ge2, D2, H2, W2, gcat2, gw[7], gb[7]);
    memcpy(gc2, gcat2, 2 * c * V2 * sizeof(double));
    for (size_t i = 0; i < 2 * c * V2; ++i) gs2[i] += gcat2[2 * c * V2 + i];
    relu_bwd(A.c2, gc2, 2 * c * V2);
    conv_bwd(&n.L[6], n.w[6], A.u2, gc2, D2, H2, W2, gu2, gw[6], gb[6]);
    up_bwd(gu2, 4 * c, D3, H3, W3, gb3);
    relu_bwd(A.b3, gb3, 4 * c * V3);
    conv_bwd(&n.L[5], n.w[5], A.a3, gb3, D3, H3, W3, ga3, gw[5], gb[5]);
    relu_bwd(A.a3, ga3, 4 * c * V3);
    conv_bwd(&n.L[4], n.w[4], A.p2, ga3, D3, H3, W3, gp2, gw[4], gb[4]);
    pool_bwd(gp2, 2 * c, D2, H2, W2, gs2);
    relu_bwd(A.s2, gs2, 2 * c * V2);
    conv_bwd(&n.L[3], n.w[3], A.a2, gs2, D2, H2, W2, ga2, gw[3], gb[3]);
    relu_bwd(A.a2, ga2, 2 * c * V2);
    conv_bwd(&n.L[2], n.w[2], A.p1, ga2, D2, H2, W2, gp1, gw[2], gb[2]);
    pool_bwd(gp1, c, D, H, W, gs1);
    relu_bwd(A.s1, gs1, c * V1);
    conv_bwd(&n.L[1], n.w[1], A.a1, gs1, D, H, W, ga1, gw[1], gb[1]);
    relu_bwd(A.a1, ga1, c * V1);
    conv_bwd(&n.L[0], n.w[0], A.inq, ga1, D, H, W, NULL, gw[0], gb[0]);

    double *tofree[] = {gh, ge1, gcat1, gu1, ge2, gcat2, gu2, gb3, ga3, gp2, gs2, ga2, gp1, gs1, ga1, gc1, gc2};
    for (size_t i = 0; i < sizeof(tofree) / sizeof(tofree[0]); ++i) free(tofree[i]);
    acts_free(&A);
    free(n.wr);
    return loss;
}
