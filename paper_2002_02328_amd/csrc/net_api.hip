// Host side of the learned warm start: the network handle, its parameters and
// Adam state, activation buffers per input shape, and the bd3mg_net_* calls
// declared in include/bd3mg.h.  Every pass is enqueued on the handle's stream.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/bd3mg.h"
#include "bd3mg_internal.h"
#include "net_internal.h"

using namespace bd3net;
using bd3mg::fail;

namespace {

constexpr int NL = 11;
constexpr uint32_t BLOB_MAGIC = 0x4e334442u;  // "BD3N"
constexpr uint32_t BLOB_VERSION = 1;
constexpr size_t PART_BYTES = 64u << 20;      // weight-gradient partials
constexpr int NWG_MAX = 1024;

struct Layer {
    int cin, cout, k;
    size_t w_off, b_off;
};

struct Acts {  // forward activations (bf16, channels last) of one input shape
    Vol v{0, 0, 0, 0};
    float *y = nullptr, *x0 = nullptr, *t = nullptr;
    bf16_t *a1 = nullptr, *s1 = nullptr, *p1 = nullptr, *a2 = nullptr, *s2 = nullptr, *p2 = nullptr;
    bf16_t *a3 = nullptr, *b3 = nullptr, *c2 = nullptr, *e2 = nullptr, *c1 = nullptr, *e1 = nullptr;
};

struct Grads {  // backward buffers of one input shape
    Vol v{0, 0, 0, 0};
    bf16_t *g9 = nullptr, *g8 = nullptr, *g7 = nullptr, *g6 = nullptr, *g5 = nullptr, *g4 = nullptr;
    bf16_t *g3 = nullptr, *g2 = nullptr, *g1 = nullptr, *g0 = nullptr;
    float *gs1p = nullptr, *gu1 = nullptr, *gs2p = nullptr, *gu2 = nullptr, *gp2 = nullptr, *gp1 = nullptr;
    double *hpart = nullptr;
};

bool same(const Vol &a, const Vol &b) { return a.nb == b.nb && a.D == b.D && a.H == b.H && a.W == b.W; }

}  // namespace

struct bd3mg_net_s {
    int levels = 3, c = 16, cin = 1;
    Layer L[NL];
    size_t nparams = 0;
    hipStream_t stream = nullptr;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    bf16_t *wk[NL] = {}, *wt[NL] = {};
    float *w0r = nullptr, *whr = nullptr;
    float *part = nullptr, *partb = nullptr;
    double *sq = nullptr;
    long long step = 0;
    Acts A;
    Grads G;
};

namespace {

template <typename T>
bd3mg_status dalloc(T **ptr, size_t count, const char *what)
{
    if (hipMalloc((void **)ptr, (count ? count : 1) * sizeof(T)) != hipSuccess)
        return fail(BD3MG_ERR_NOMEM, "device allocation failed: %s (%zu bytes)", what, count * sizeof(T));
    return BD3MG_OK;
}

template <typename T>
void dfree(T *&ptr)
{
    if (ptr) (void)hipFree((void *)ptr);
    ptr = nullptr;
}

void free_acts(Acts &A)
{
    dfree(A.y), dfree(A.x0), dfree(A.t);
    bf16_t **b[] = {&A.a1, &A.s1, &A.p1, &A.a2, &A.s2, &A.p2, &A.a3, &A.b3, &A.c2, &A.e2, &A.c1, &A.e1};
    for (auto q : b) dfree(*q);
    A.v = Vol{0, 0, 0, 0};
}

void free_grads(Grads &G)
{
    bf16_t **b[] = {&G.g9, &G.g8, &G.g7, &G.g6, &G.g5, &G.g4, &G.g3, &G.g2, &G.g1, &G.g0};
    for (auto q : b) dfree(*q);
    float **f[] = {&G.gs1p, &G.gu1, &G.gs2p, &G.gu2, &G.gp2, &G.gp1};
    for (auto q : f) dfree(*q);
    dfree(G.hpart);
    G.v = Vol{0, 0, 0, 0};
}

bd3mg_status ensure_acts(bd3mg_net n, const Vol &v)
{
    if (same(n->A.v, v)) return BD3MG_OK;
    HIP_TRY(hipStreamSynchronize(n->stream));
    free_acts(n->A);
    const int c = n->c;
    const size_t V1 = v.voxels(), V2 = v.half().voxels(), V3 = v.half().half().voxels();
    Acts &A = n->A;
    ST_TRY(dalloc(&A.y, V1, "input"));
    ST_TRY(dalloc(&A.x0, V1, "output"));
    ST_TRY(dalloc(&A.t, V1, "target"));
    ST_TRY(dalloc(&A.a1, c * V1, "a1"));
    ST_TRY(dalloc(&A.s1, c * V1, "s1"));
    ST_TRY(dalloc(&A.p1, c * V2, "p1"));
    ST_TRY(dalloc(&A.a2, 2 * c * V2, "a2"));
    ST_TRY(dalloc(&A.s2, 2 * c * V2, "s2"));
    ST_TRY(dalloc(&A.p2, 2 * c * V3, "p2"));
    ST_TRY(dalloc(&A.a3, 4 * c * V3, "a3"));
    ST_TRY(dalloc(&A.b3, 4 * c * V3, "b3"));
    ST_TRY(dalloc(&A.c2, 2 * c * V2, "c2"));
    ST_TRY(dalloc(&A.e2, 2 * c * V2, "e2"));
    ST_TRY(dalloc(&A.c1, c * V1, "c1"));
    ST_TRY(dalloc(&A.e1, c * V1, "e1"));
    A.v = v;
    return BD3MG_OK;
}

bd3mg_status ensure_grads(bd3mg_net n, const Vol &v)
{
    if (same(n->G.v, v)) return BD3MG_OK;
    HIP_TRY(hipStreamSynchronize(n->stream));
    free_grads(n->G);
    const int c = n->c;
    const size_t V1 = v.voxels(), V2 = v.half().voxels(), V3 = v.half().half().voxels();
    Grads &G = n->G;
    ST_TRY(dalloc(&G.g9, c * V1, "g9"));
    ST_TRY(dalloc(&G.g8, c * V1, "g8"));
    ST_TRY(dalloc(&G.gs1p, c * V1, "gs1p"));
    ST_TRY(dalloc(&G.gu1, 2 * c * V1, "gu1"));
    ST_TRY(dalloc(&G.g7, 2 * c * V2, "g7"));
    ST_TRY(dalloc(&G.g6, 2 * c * V2, "g6"));
    ST_TRY(dalloc(&G.gs2p, 2 * c * V2, "gs2p"));
    ST_TRY(dalloc(&G.gu2, 4 * c * V2, "gu2"));
    ST_TRY(dalloc(&G.g5, 4 * c * V3, "g5"));
    ST_TRY(dalloc(&G.g4, 4 * c * V3, "g4"));
    ST_TRY(dalloc(&G.gp2, 2 * c * V3, "gp2"));
    ST_TRY(dalloc(&G.g3, 2 * c * V2, "g3"));
    ST_TRY(dalloc(&G.g2, 2 * c * V2, "g2"));
    ST_TRY(dalloc(&G.gp1, c * V2, "gp1"));
    ST_TRY(dalloc(&G.g1, c * V1, "g1"));
    ST_TRY(dalloc(&G.g0, c * V1, "g0"));
    ST_TRY(dalloc(&G.hpart, ((V1 + NTH - 1) / NTH) * 18, "head partials"));
    G.v = v;
    return BD3MG_OK;
}

// bf16 copies of the weights in the layouts of the forward and data-gradient
// products, after every change of the float parameters.
bd3mg_status repack(bd3mg_net n)
{
    for (int i = 1; i < NL - 1; ++i) {
        HIP_TRY(pack_fwd(n->L[i].cin, n->L[i].cout, n->p + n->L[i].w_off, n->wk[i], n->stream));
        HIP_TRY(pack_bwd(n->L[i].cin, n->L[i].cout, n->p + n->L[i].w_off, n->wt[i], n->stream));
    }
    HIP_TRY(round_bf16(n->p + n->L[0].w_off, n->w0r, n->L[0].cout * 27, n->stream));
    HIP_TRY(round_bf16(n->p + n->L[NL - 1].w_off, n->whr, n->L[NL - 1].cin, n->stream));
    return BD3MG_OK;
}

bd3mg_status check_shape(bd3mg_net n, int nb, int nx, int ny, int nz)
{
    if (!n) return fail(BD3MG_ERR_ARG, "null network handle");
    if (nb < 1 || nx < 4 || ny < 4 || nz < 4)
        return fail(BD3MG_ERR_ARG, "batch must be >= 1 and every side >= 4");
    if (nx % 4 || ny % 4 || nz % 4)
        return fail(BD3MG_ERR_ARG, "volume sides must be multiples of 4 (two 2x2x2 poolings)");
    if ((size_t)nb * nx * ny * nz > ((size_t)1 << 31))
        return fail(BD3MG_ERR_ARG, "batch too large (more than 2^31 voxels)");
    return BD3MG_OK;
}

bd3mg_status forward(bd3mg_net n)
{
    Acts &A = n->A;
    const Vol v1 = A.v, v2 = v1.half(), v3 = v2.half();
    const Layer *L = n->L;
    const float *P = n->p;
    hipStream_t st = n->stream;
    const ConvIn none{nullptr, nullptr, 0};
    (void)none;
    HIP_TRY(conv0_fwd(v1, A.y, n->w0r, P + L[0].b_off, A.a1, st));
    HIP_TRY(conv3(16, 16, SRC_PLAIN, 0, v1, ConvIn{A.a1, nullptr, 0}, n->wk[1], P + L[1].b_off, 0, nullptr, A.s1, nullptr, st));
    HIP_TRY(pool_fwd(v1, 16, A.s1, A.p1, st));
    HIP_TRY(conv3(16, 32, SRC_PLAIN, 0, v2, ConvIn{A.p1, nullptr, 0}, n->wk[2], P + L[2].b_off, 0, nullptr, A.a2, nullptr, st));
    HIP_TRY(conv3(32, 32, SRC_PLAIN, 0, v2, ConvIn{A.a2, nullptr, 0}, n->wk[3], P + L[3].b_off, 0, nullptr, A.s2, nullptr, st));
    HIP_TRY(pool_fwd(v2, 32, A.s2, A.p2, st));
    HIP_TRY(conv3(32, 64, SRC_PLAIN, 0, v3, ConvIn{A.p2, nullptr, 0}, n->wk[4], P + L[4].b_off, 0, nullptr, A.a3, nullptr, st));
    HIP_TRY(conv3(64, 64, SRC_PLAIN, 0, v3, ConvIn{A.a3, nullptr, 0}, n->wk[5], P + L[5].b_off, 0, nullptr, A.b3, nullptr, st));
    HIP_TRY(conv3(64, 32, SRC_UP, 0, v2, ConvIn{A.b3, nullptr, 0}, n->wk[6], P + L[6].b_off, 0, nullptr, A.c2, nullptr, st));
    HIP_TRY(conv3(64, 32, SRC_CAT, 0, v2, ConvIn{A.c2, A.s2, 32}, n->wk[7], P + L[7].b_off, 0, nullptr, A.e2, nullptr, st));
    HIP_TRY(conv3(32, 16, SRC_UP, 0, v1, ConvIn{A.e2, nullptr, 0}, n->wk[8], P + L[8].b_off, 0, nullptr, A.c1, nullptr, st));
    HIP_TRY(conv3(32, 16, SRC_CAT, 0, v1, ConvIn{A.c1, A.s1, 16}, n->wk[9], P + L[9].b_off, 0, nullptr, A.e1, nullptr, st));
    HIP_TRY(head_fwd(v1, A.e1, A.y, n->whr, P + L[10].b_off, A.x0, st));
    return BD3MG_OK;
}

// Weight and bias gradient of layer i from its pre-activation gradient g and input.
bd3mg_status layer_wgrad(bd3mg_net n, int i, int src, const Vol &v, const bf16_t *g, ConvIn in)
{
    const Layer &l = n->L[i];
    const int ne = l.cout * l.cin * 27;
    int cap = (int)(PART_BYTES / ((size_t)ne * sizeof(float)));
    cap = cap < NWG_MAX ? cap : NWG_MAX;
    int nwg = 0;
    HIP_TRY(wgrad3(l.cin, l.cout, src, v, g, in, n->part, n->partb, cap, &nwg, n->stream));
    HIP_TRY(wreduce(n->part, nwg, ne, n->g + l.w_off, n->partb, l.cout, n->g + l.b_off, n->stream));
    return BD3MG_OK;
}

// Gradient of the mean squared error of the last forward pass against A.t,
// into n->g; the sum of squared errors is left in n->sq.
bd3mg_status backward(bd3mg_net n)
{
    Acts &A = n->A;
    Grads &G = n->G;
    const Vol v1 = A.v, v2 = v1.half(), v3 = v2.half();
    hipStream_t st = n->stream;
    int nh = 0;
    HIP_TRY(head_bwd(v1, A.e1, A.x0, A.t, n->whr, G.g9, G.hpart, &nh, st));
    HIP_TRY(head_reduce(G.hpart, nh, n->g + n->L[10].w_off, n->sq, st));

    ST_TRY(layer_wgrad(n, 9, SRC_CAT, v1, G.g9, ConvIn{A.c1, A.s1, 16}));
    HIP_TRY(conv3(16, 32, SRC_PLAIN, 1, v1, ConvIn{G.g9, nullptr, 0}, n->wt[9], nullptr, 16, A.c1, G.g8, G.gs1p, st));
    ST_TRY(layer_wgrad(n, 8, SRC_UP, v1, G.g8, ConvIn{A.e2, nullptr, 0}));
    HIP_TRY(conv3(16, 32, SRC_PLAIN, 1, v1, ConvIn{G.g8, nullptr, 0}, n->wt[8], nullptr, 0, nullptr, nullptr, G.gu1, st));
    HIP_TRY(up_bwd(v1, 32, G.gu1, A.e2, G.g7, st));
    ST_TRY(layer_wgrad(n, 7, SRC_CAT, v2, G.g7, ConvIn{A.c2, A.s2, 32}));
    HIP_TRY(conv3(32, 64, SRC_PLAIN, 1, v2, ConvIn{G.g7, nullptr, 0}, n->wt[7], nullptr, 32, A.c2, G.g6, G.gs2p, st));
    ST_TRY(layer_wgrad(n, 6, SRC_UP, v2, G.g6, ConvIn{A.b3, nullptr, 0}));
    HIP_TRY(conv3(32, 64, SRC_PLAIN, 1, v2, ConvIn{G.g6, nullptr, 0}, n->wt[6], nullptr, 0, nullptr, nullptr, G.gu2, st));
    HIP_TRY(up_bwd(v2, 64, G.gu2, A.b3, G.g5, st));
    ST_TRY(layer_wgrad(n, 5, SRC_PLAIN, v3, G.g5, ConvIn{A.a3, nullptr, 0}));
    HIP_TRY(conv3(64, 64, SRC_PLAIN, 1, v3, ConvIn{G.g5, nullptr, 0}, n->wt[5], nullptr, 64, A.a3, G.g4, nullptr, st));
    ST_TRY(layer_wgrad(n, 4, SRC_PLAIN, v3, G.g4, ConvIn{A.p2, nullptr, 0}));
    HIP_TRY(conv3(64, 32, SRC_PLAIN, 1, v3, ConvIn{G.g4, nullptr, 0}, n->wt[4], nullptr, 0, nullptr, nullptr, G.gp2, st));
    HIP_TRY(pool_bwd(v2, 32, G.gs2p, G.gp2, A.s2, G.g3, st));
    ST_TRY(layer_wgrad(n, 3, SRC_PLAIN, v2, G.g3, ConvIn{A.a2, nullptr, 0}));
    HIP_TRY(conv3(32, 32, SRC_PLAIN, 1, v2, ConvIn{G.g3, nullptr, 0}, n->wt[3], nullptr, 32, A.a2, G.g2, nullptr, st));
    ST_TRY(layer_wgrad(n, 2, SRC_PLAIN, v2, G.g2, ConvIn{A.p1, nullptr, 0}));
    HIP_TRY(conv3(32, 16, SRC_PLAIN, 1, v2, ConvIn{G.g2, nullptr, 0}, n->wt[2], nullptr, 0, nullptr, nullptr, G.gp1, st));
    HIP_TRY(pool_bwd(v1, 16, G.gs1p, G.gp1, A.s1, G.g1, st));
    ST_TRY(layer_wgrad(n, 1, SRC_PLAIN, v1, G.g1, ConvIn{A.a1, nullptr, 0}));
    HIP_TRY(conv3(16, 16, SRC_PLAIN, 1, v1, ConvIn{G.g1, nullptr, 0}, n->wt[1], nullptr, 16, A.a1, G.g0, nullptr, st));
    {
        int nwg = 0;
        const Layer &l = n->L[0];
        HIP_TRY(conv0_wgrad(v1, G.g0, A.y, n->part, n->partb, NWG_MAX, &nwg, st));
        HIP_TRY(wreduce(n->part, nwg, l.cout * 27, n->g + l.w_off, n->partb, l.cout, n->g + l.b_off, st));
    }
    return BD3MG_OK;
}

bd3mg_status load_pair(bd3mg_net n, int nb, int nx, int ny, int nz, const float *y, const float *t, int on_device)
{
    ST_TRY(check_shape(n, nb, nx, ny, nz));
    if (!y) return fail(BD3MG_ERR_ARG, "null input");
    const Vol v{nb, nz, ny, nx};
    ST_TRY(ensure_acts(n, v));
    const size_t bytes = v.voxels() * sizeof(float);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(hipMemcpyAsync(n->A.y, y, bytes, kind, n->stream));
    if (t) HIP_TRY(hipMemcpyAsync(n->A.t, t, bytes, kind, n->stream));
    return BD3MG_OK;
}

}  // namespace

extern "C" {

bd3mg_status bd3mg_net_create(int levels, int base_channels, int in_channels, bd3mg_net *out)
{
    if (!out) return fail(BD3MG_ERR_ARG, "null output handle");
    *out = nullptr;
    if (levels != 3 || base_channels != 16 || in_channels != 1)
        return fail(BD3MG_ERR_ARG, "supported network: 3 levels, 16 base channels, 1 input channel");
    bd3mg_net n = new (std::nothrow) bd3mg_net_s;
    if (!n) return fail(BD3MG_ERR_NOMEM, "handle");
    const int c = base_channels;
    const int spec[NL][3] = {{in_channels, c, 3}, {c, c, 3},         {c, 2 * c, 3},     {2 * c, 2 * c, 3},
                             {2 * c, 4 * c, 3},   {4 * c, 4 * c, 3}, {4 * c, 2 * c, 3}, {4 * c, 2 * c, 3},
                             {2 * c, c, 3},       {2 * c, c, 3},     {c, 1, 1}};
    size_t off = 0;
    for (int i = 0; i < NL; ++i) {
        Layer &l = n->L[i];
        l.cin = spec[i][0];
        l.cout = spec[i][1];
        l.k = spec[i][2];
        l.w_off = off;
        l.b_off = off + (size_t)l.cout * l.cin * l.k * l.k * l.k;
        off = l.b_off + l.cout;
    }
    n->nparams = off;
    auto bail = [&](bd3mg_status st) {
        bd3mg_net_destroy(n);
        return st;
    };
    if (hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(BD3MG_ERR_HIP, "stream creation failed"));
    bd3mg_status st = BD3MG_OK;
    if ((st = dalloc(&n->p, off, "parameters")) || (st = dalloc(&n->g, off, "gradient")) ||
        (st = dalloc(&n->m, off, "Adam m")) || (st = dalloc(&n->v, off, "Adam v")) ||
        (st = dalloc(&n->w0r, 16 * 27, "first layer")) || (st = dalloc(&n->whr, 16, "head")) ||
        (st = dalloc(&n->part, PART_BYTES / sizeof(float), "partials")) ||
        (st = dalloc(&n->partb, (size_t)NWG_MAX * 64, "bias partials")) || (st = dalloc(&n->sq, 1, "loss")))
        return bail(st);
    for (int i = 1; i < NL - 1; ++i) {
        const Layer &l = n->L[i];
        if ((st = dalloc(&n->wk[i], (size_t)l.cout * kpad(l.cin), "packed weights")) ||
            (st = dalloc(&n->wt[i], (size_t)l.cin * kpad(l.cout), "packed weights")))
            return bail(st);
    }
    if (hipMemsetAsync(n->p, 0, off * sizeof(float), n->stream) != hipSuccess ||
        hipMemsetAsync(n->m, 0, off * sizeof(float), n->stream) != hipSuccess ||
        hipMemsetAsync(n->v, 0, off * sizeof(float), n->stream) != hipSuccess)
        return bail(fail(BD3MG_ERR_HIP, "clearing parameters failed"));
    if ((st = repack(n)) != BD3MG_OK) return bail(st);
    if (hipStreamSynchronize(n->stream) != hipSuccess) return bail(fail(BD3MG_ERR_HIP, "stream sync failed"));
    *out = n;
    return BD3MG_OK;
}

bd3mg_status bd3mg_net_destroy(bd3mg_net n)
{
    if (!n) return BD3MG_OK;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    free_acts(n->A);
    free_grads(n->G);
    dfree(n->p), dfree(n->g), dfree(n->m), dfree(n->v), dfree(n->w0r), dfree(n->whr);
    dfree(n->part), dfree(n->partb), dfree(n->sq);
    for (int i = 0; i < NL; ++i) dfree(n->wk[i]), dfree(n->wt[i]);
    if (n->stream) (void)hipStreamDestroy(n->stream);
    delete n;
    return BD3MG_OK;
}

bd3mg_status bd3mg_net_num_params(bd3mg_net n, size_t *count)
{
    if (!n || !count) return fail(BD3MG_ERR_ARG, "null argument");
    *count = n->nparams;
    return BD3MG_OK;
}

bd3mg_status bd3mg_net_set_params(bd3mg_net n, const float *params, size_t count)
{
    if (!n || !params) return fail(BD3MG_ERR_ARG, "null argument");
    if (count != n->nparams) return fail(BD3MG_ERR_ARG, "expected %zu parameters, got %zu", n->nparams, count);
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(params[i])) return fail(BD3MG_ERR_ARG, "parameter %zu is not finite", i);
    HIP_TRY(hipMemcpyAsync(n->p, params, count * sizeof(float), hipMemcpyHostToDevice, n->stream));
    HIP_TRY(hipMemsetAsync(n->m, 0, count * sizeof(float), n->stream));
    HIP_TRY(hipMemsetAsync(n->v, 0, count * sizeof(float), n->stream));
    n->step = 0;
    ST_TRY(repack(n));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return BD3MG_OK;
}

bd3mg_status bd3mg_net_get_params(bd3mg_net n, float *params, size_t count)
{
    if (!n || !params) return fail(BD3MG_ERR_ARG, "null argument");
    if (count != n->nparams) return fail(BD3MG_ERR_ARG, "expected %zu parameters, got %zu", n->nparams, count);
    HIP_TRY(hipMemcpyAsync(params, n->p, count * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return BD3MG_OK;
}

bd3mg_status bd3mg_net_save(bd3mg_net n, void *blob, size_t *bytes)
{
    if (!n || !bytes) return fail(BD3MG_ERR_ARG, "null argument");
    const size_t need = 6 * sizeof(uint32_t) + n->nparams * sizeof(float);
    if (!blob) {
        *bytes = need;
        return BD3MG_OK;
    }
    if (*bytes < need) return fail(BD3MG_ERR_ARG, "blob needs %zu bytes", need);
    uint32_t hdr[6] = {BLOB_MAGIC, BLOB_VERSION, (uint32_t)n->levels, (uint32_t)n->c, (uint32_t)n->cin,
                       (uint32_t)n->nparams};
    std::memcpy(blob, hdr, sizeof(hdr));
    ST_TRY(bd3mg_net_get_params(n, (float *)((char *)blob + sizeof(hdr)), n->nparams));
    *bytes = need;
    return BD3MG_OK;
}

bd3mg_status bd3mg_net_load(bd3mg_net n, const void *blob, size_t bytes)
{
    if (!n || !blob) return fail(BD3MG_ERR_ARG, "null argument");
    uint32_t hdr[6];
    if (bytes < sizeof(hdr)) return fail(BD3MG_ERR_ARG, "blob too short");
    std::memcpy(hdr, blob, sizeof(hdr));
    if (hdr[0] != BLOB_MAGIC || hdr[1] != BLOB_VERSION) return fail(BD3MG_ERR_ARG, "not a network blob");
    if ((int)hdr[2] != n->levels || (int)hdr[3] != n->c || (int)hdr[4] != n->cin || hdr[5] != n->nparams)
        return fail(BD3MG_ERR_ARG, "blob is for another network shape");
    if (bytes != sizeof(hdr) + n->nparams * sizeof(float)) return fail(BD3MG_ERR_ARG, "blob size mismatch");
    std::vector<float> p(n->nparams);
    std::memcpy(p.data(), (const char *)blob + sizeof(hdr), n->nparams * sizeof(float));
    return bd3mg_net_set_params(n, p.data(), n->nparams);
}

bd3mg_status bd3mg_net_forward(bd3mg_net n, int nb, int nx, int ny, int nz, const float *y, float *x0,
                               int on_device)
{
    if (!x0) return fail(BD3MG_ERR_ARG, "null output");
    ST_TRY(load_pair(n, nb, nx, ny, nz, y, nullptr, on_device));
    ST_TRY(forward(n));
    HIP_TRY(hipMemcpyAsync(x0, n->A.x0, n->A.v.voxels() * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    return BD3MG_OK;
}

bd3mg_status bd3mg_net_infer(bd3mg_net n, bd3mg_problem p)
{
    if (!n) return fail(BD3MG_ERR_ARG, "null network handle");
    bd3mg::ProblemView pv;
    ST_TRY(bd3mg::problem_view(p, &pv));
    if (!pv.data_set) return fail(BD3MG_ERR_STATE, "the problem has no data");
    ST_TRY(check_shape(n, 1, pv.nx, pv.ny, pv.nz));
    const Vol v{1, pv.nz, pv.ny, pv.nx};
    ST_TRY(ensure_acts(n, v));
    HIP_TRY(hipStreamSynchronize(pv.stream));
    const size_t N = v.voxels();
    if (pv.prec == BD3MG_FP32) {
        HIP_TRY(hipMemcpyAsync(n->A.y, pv.y, N * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    } else {
        HIP_TRY(f64_to_f32((const double *)pv.y, n->A.y, N, n->stream));
    }
    ST_TRY(forward(n));
    if (pv.prec == BD3MG_FP32) {
        HIP_TRY(hipStreamSynchronize(n->stream));
        return bd3mg_set_x0(p, n->A.x0, 1);
    }
    double *tmp = nullptr;
    ST_TRY(dalloc(&tmp, N, "start point"));
    bd3mg_status st = BD3MG_OK;
    if (f32_to_f64(n->A.x0, tmp, N, n->stream) != hipSuccess || hipStreamSynchronize(n->stream) != hipSuccess)
        st = fail(BD3MG_ERR_HIP, "start point conversion failed");
    if (st == BD3MG_OK) st = bd3mg_set_x0(p, tmp, 1);
    dfree(tmp);
    return st;
}

bd3mg_status bd3mg_net_grad(bd3mg_net n, int nb, int nx, int ny, int nz, const float *y, const float *xstar,
                            int on_device, float *grad, double *loss)
{
    if (!xstar || !grad) return fail(BD3MG_ERR_ARG, "null argument");
    ST_TRY(load_pair(n, nb, nx, ny, nz, y, xstar, on_device));
    ST_TRY(ensure_grads(n, n->A.v));
    ST_TRY(forward(n));
    ST_TRY(backward(n));
    double sq = 0.0;
    HIP_TRY(hipMemcpyAsync(grad, n->g, n->nparams * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipMemcpyAsync(&sq, n->sq, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
    if (loss) *loss = sq / (double)n->A.v.voxels();
    return BD3MG_OK;
}

bd3mg_status bd3mg_net_train_step(bd3mg_net n, int nb, int nx, int ny, int nz, const float *y,
                                  const float *xstar, int on_device, float lr, double *loss)
{
    if (!xstar) return fail(BD3MG_ERR_ARG, "null target");
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(BD3MG_ERR_ARG, "learning rate must be positive");
    ST_TRY(load_pair(n, nb, nx, ny, nz, y, xstar, on_device));
    ST_TRY(ensure_grads(n, n->A.v));
    ST_TRY(forward(n));
    ST_TRY(backward(n));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    n->step += 1;
    const float bc1 = (float)(1.0 - std::pow((double)b1, (double)n->step));
    const float bc2 = (float)(1.0 - std::pow((double)b2, (double)n->step));
    HIP_TRY(adam(n->p, n->g, n->m, n->v, n->nparams, lr, b1, b2, eps, bc1, bc2, n->stream));
    ST_TRY(repack(n));
    if (loss) {
        double sq = 0.0;
        HIP_TRY(hipMemcpyAsync(&sq, n->sq, sizeof(double), hipMemcpyDeviceToHost, n->stream));
        HIP_TRY(hipStreamSynchronize(n->stream));
        *loss = sq / (double)n->A.v.voxels();
    } else {
        HIP_TRY(hipStreamSynchronize(n->stream));
    }
    return BD3MG_OK;
}

}  // extern "C"
