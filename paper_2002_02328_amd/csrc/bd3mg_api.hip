// Host side of libbd3mg: problem state, block schedule, and the C interface
// declared in include/bd3mg.h.
//
// One BD3MG sweep (every block updated once, Sec. 2.3 boxes "Master" and
// "Worker") runs as, for each colour of blocks:
//   gradient pass  (g on the blocks, <g,g>, <g,dp>, <dp,dp>)
//   direction pass (H d1, H d2 and the majorant inner products)
//   solve          (2x2 system and step coefficients, per block, in double)
//   update pass    (x += d', dp = d', r += H d')
// all enqueued on the problem's stream; the host only waits at stop checks.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bd3mg.h"
#include "bd3mg_internal.h"

using namespace bd3mg;

namespace {

thread_local std::string g_err;

bd3mg_status fail(bd3mg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(BD3MG_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                        __FILE__, __LINE__);                                                 \
    } while (0)

#define ST_TRY(expr)                                   \
    do {                                               \
        bd3mg_status s_ = (expr);                      \
        if (s_ != BD3MG_OK) return s_;                 \
    } while (0)

// Whole-volume passes split the slices into chunks of this many slices.
constexpr int CHUNK = 8;

}  // namespace

struct bd3mg_problem_s {
    int nx = 0, ny = 0, nz = 0, prec = 0;
    size_t N = 0, esz = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    Geom geom{};
    Params prm{0.0, 1.0, 0.0, 0.0, 0.0, 1.0};

    // PSF
    bool psf_set = false;
    int kx = 0, ky = 0, kz = 0;
    void *d_gx = nullptr, *d_gy = nullptr, *d_gz = nullptr;

    // volumes (storage type)
    void *x = nullptr, *y = nullptr, *r = nullptr, *g = nullptr, *dpb[2] = {nullptr, nullptr};
    void *tmp[3] = {nullptr, nullptr, nullptr};
    int cur = 0;  // dpb[cur] holds every block's last step
    bool data_set = false, x_set = false, r_stale = true;

    // blocks and schedule
    bool blocks_set = false, sched_dirty = true;
    int schedule = BD3MG_SCHED_COLORED;
    std::vector<int> nsl, z0, order, color;
    int ncolors = 0;
    std::vector<int> col_off, col_cnt;  // segments of each colour in d_segs
    Segment *d_segs = nullptr;
    int nseg_alloc = 0;
    Segment *d_chunks = nullptr;
    int nchunks = 0;

    // reductions
    double *d_partials = nullptr;
    size_t partials_cap = 0;  // doubles
    double *d_u = nullptr, *d_info = nullptr, *d_eval = nullptr;
    int nblocks_alloc = 0;

    double gnorm_ref = 0.0;
    bool gnorm_ref_valid = false;

    long long sweeps_done = 0;  // sweeps since x^0 (drives the residual refresh)
    long long refresh_every = 0;

    // profiling: event pairs of the launches not yet folded into the totals
    bool profile = false;
    struct Pending {
        int kind;
        double bytes;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    long long prof_launches[BD3MG_K_COUNT] = {0, 0, 0, 0, 0};
    double prof_ms[BD3MG_K_COUNT] = {0, 0, 0, 0, 0};
    double prof_bytes[BD3MG_K_COUNT] = {0, 0, 0, 0, 0};
    std::vector<double> color_bytes;  // algorithmic bytes of each colour's passes, [ncolors][4]
};

namespace {

template <typename T>
DevState<T> dev_state(bd3mg_problem p)
{
    DevState<T> s;
    s.x = (T *)p->x;
    s.y = (T *)p->y;
    s.r = (T *)p->r;
    s.g = (T *)p->g;
    s.dp[0] = (T *)p->dpb[p->cur];
    s.dp[1] = (T *)p->dpb[p->cur ^ 1];
    s.gx = (const T *)p->d_gx;
    s.gy = (const T *)p->d_gy;
    s.gz = (const T *)p->d_gz;
    return s;
}

bd3mg_status check_finite(const double *v, size_t n, const char *what)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return fail(BD3MG_ERR_ARG, "%s[%zu] is not finite", what, i);
    return BD3MG_OK;
}

hipEvent_t pool_event(bd3mg_problem p)
{
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Record the start of a profiled launch (no-op unless profiling).
bd3mg_status prof_begin(bd3mg_problem p, int kind, double bytes)
{
    if (!p->profile) return BD3MG_OK;
    bd3mg_problem_s::Pending q{kind, bytes, pool_event(p), pool_event(p)};
    if (!q.a || !q.b) return fail(BD3MG_ERR_HIP, "event creation failed");
    HIP_TRY(hipEventRecord(q.a, p->stream));
    p->pending.push_back(q);
    return BD3MG_OK;
}

bd3mg_status prof_end(bd3mg_problem p)
{
    if (!p->profile) return BD3MG_OK;
    HIP_TRY(hipEventRecord(p->pending.back().b, p->stream));
    return BD3MG_OK;
}

// Fold completed launches into the totals (waits for the stream).
bd3mg_status prof_collect(bd3mg_problem p)
{
    if (p->pending.empty()) return BD3MG_OK;
    HIP_TRY(hipStreamSynchronize(p->stream));
    for (auto &q : p->pending) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, q.a, q.b));
        p->prof_launches[q.kind] += 1;
        p->prof_ms[q.kind] += ms;
        p->prof_bytes[q.kind] += q.bytes;
        p->event_pool.push_back(q.a);
        p->event_pool.push_back(q.b);
    }
    p->pending.clear();
    return BD3MG_OK;
}

// Algorithmic bytes of the passes of one colour (each element a pass must
// read or write counted once): gradient pass reads r on S +- r_z and x, dp on
// S, writes g on S; direction pass reads g, dp and x on S; solve reads the
// partial sums; update pass reads g, dp, x on S and r on S +- r_z, writes x,
// dp on S and r on S +- r_z.
void color_bytes(bd3mg_problem p)
{
    const int nb = (int)p->nsl.size();
    const double A = (double)p->nx * p->ny * p->esz;
    const int rz = p->kz / 2;
    p->color_bytes.assign((size_t)p->ncolors * 4, 0.0);
    std::vector<char> inhalo(p->nz);
    for (int c = 0; c < p->ncolors; ++c) {
        std::fill(inhalo.begin(), inhalo.end(), 0);
        double sl = 0.0, nblk = 0.0;
        for (int b = 0; b < nb; ++b) {
            if (p->color[b] != c) continue;
            sl += p->nsl[b];
            nblk += 1.0;
            for (int k = std::max(0, p->z0[b] - rz); k < std::min(p->nz, p->z0[b] + p->nsl[b] + rz); ++k)
                inhalo[k] = 1;
        }
        double h = 0.0;
        for (int k = 0; k < p->nz; ++k) h += inhalo[k];
        double *cb = &p->color_bytes[(size_t)c * 4];
        cb[0] = A * (h + 3.0 * sl);
        cb[1] = A * 3.0 * sl;
        cb[2] = nblk * p->geom.ntx * p->geom.nty * NQ * sizeof(double);
        cb[3] = A * (5.0 * sl + 2.0 * h);
    }
}

bd3mg_status ensure_partials(bd3mg_problem p, size_t doubles)
{
    if (doubles <= p->partials_cap) return BD3MG_OK;
    if (p->d_partials) HIP_TRY(hipFree(p->d_partials));
    p->d_partials = nullptr;
    p->partials_cap = 0;
    if (hipMalloc(&p->d_partials, doubles * sizeof(double)) != hipSuccess)
        return fail(BD3MG_ERR_NOMEM, "partial-sum buffer of %zu doubles", doubles);
    p->partials_cap = doubles;
    return BD3MG_OK;
}

bd3mg_status ensure_tmp(bd3mg_problem p, int count)
{
    for (int i = 0; i < count; ++i)
        if (!p->tmp[i] && hipMalloc(&p->tmp[i], p->N * p->esz) != hipSuccess)
            return fail(BD3MG_ERR_NOMEM, "scratch volume of %zu bytes", p->N * p->esz);
    return BD3MG_OK;
}

// Upload a volume of the storage type from host or device memory.
bd3mg_status upload(bd3mg_problem p, void *dst, const void *src, int on_device)
{
    HIP_TRY(hipMemcpyAsync(dst, src, p->N * p->esz,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return BD3MG_OK;
}

bd3mg_status download(bd3mg_problem p, void *dst, const void *src, int on_device)
{
    HIP_TRY(hipMemcpyAsync(dst, src, p->N * p->esz,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return BD3MG_OK;
}

bd3mg_status zero_steps(bd3mg_problem p)
{
    HIP_TRY(hipMemsetAsync(p->dpb[0], 0, p->N * p->esz, p->stream));
    HIP_TRY(hipMemsetAsync(p->dpb[1], 0, p->N * p->esz, p->stream));
    p->cur = 0;
    return BD3MG_OK;
}

// Greedy colouring in z order: block b takes the smallest colour none of whose
// earlier members is closer than min_gap slices.  Same-colour blocks then read
// and write disjoint data (the residual on S +- r_z, the iterate on S +- 1 when
// kappa > 0), so updating them together equals updating them in sequence.
void color_blocks(bd3mg_problem p)
{
    const int nb = (int)p->nsl.size();
    p->color.assign(nb, 0);
    p->order.clear();
    if (p->schedule == BD3MG_SCHED_SEQUENTIAL) {
        for (int b = 0; b < nb; ++b) p->color[b] = b;
        p->ncolors = nb;
    } else {
        const int rz = p->kz / 2;
        const int min_gap = std::max(2 * rz, p->prm.kappa > 0.0 ? 1 : 0);
        int nc = 0;
        for (int b = 0; b < nb; ++b) {
            int c = 0;
            for (;; ++c) {
                bool ok = true;
                for (int e = b - 1; e >= 0 && ok; --e)
                    if (p->color[e] == c && p->z0[b] - (p->z0[e] + p->nsl[e]) < min_gap) ok = false;
                if (ok) break;
            }
            p->color[b] = c;
            nc = std::max(nc, c + 1);
        }
        p->ncolors = nc;
    }
    for (int c = 0; c < p->ncolors; ++c)
        for (int b = 0; b < nb; ++b)
            if (p->color[b] == c) p->order.push_back(b);
}

bd3mg_status build_schedule(bd3mg_problem p)
{
    if (!p->sched_dirty) return BD3MG_OK;
    if (!p->blocks_set) return fail(BD3MG_ERR_STATE, "blocks are not set");
    if (!p->psf_set) return fail(BD3MG_ERR_STATE, "the PSF is not set (the colouring needs r_z)");
    color_blocks(p);
    const int nb = (int)p->nsl.size();
    std::vector<Segment> segs;
    p->col_off.assign(p->ncolors, 0);
    p->col_cnt.assign(p->ncolors, 0);
    int q = 0;
    for (int c = 0; c < p->ncolors; ++c) {
        p->col_off[c] = (int)segs.size();
        while (q < nb && p->color[p->order[q]] == c) {
            const int b = p->order[q++];
            segs.push_back(Segment{p->z0[b], p->nsl[b], b, 0});
        }
        p->col_cnt[c] = (int)segs.size() - p->col_off[c];
    }
    // single-block segments for bd3mg_block_step follow, one per block
    for (int b = 0; b < nb; ++b) segs.push_back(Segment{p->z0[b], p->nsl[b], b, 0});
    if ((int)segs.size() > p->nseg_alloc) {
        if (p->d_segs) HIP_TRY(hipFree(p->d_segs));
        p->d_segs = nullptr;
        if (hipMalloc(&p->d_segs, segs.size() * sizeof(Segment)) != hipSuccess)
            return fail(BD3MG_ERR_NOMEM, "segment table");
        p->nseg_alloc = (int)segs.size();
    }
    HIP_TRY(hipMemcpyAsync(p->d_segs, segs.data(), segs.size() * sizeof(Segment),
                           hipMemcpyHostToDevice, p->stream));
    if (nb > p->nblocks_alloc) {
        if (p->d_u) HIP_TRY(hipFree(p->d_u));
        if (p->d_info) HIP_TRY(hipFree(p->d_info));
        p->d_u = p->d_info = nullptr;
        if (hipMalloc(&p->d_u, 2 * nb * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->d_info, 8 * nb * sizeof(double)) != hipSuccess)
            return fail(BD3MG_ERR_NOMEM, "per-block coefficients");
        p->nblocks_alloc = nb;
    }
    int maxc = 1;
    for (int c = 0; c < p->ncolors; ++c) maxc = std::max(maxc, p->col_cnt[c]);
    const size_t slots = (size_t)p->geom.ntx * p->geom.nty;
    ST_TRY(ensure_partials(p, std::max(slots * maxc * NQ, slots * p->nchunks * NE)));
    HIP_TRY(hipStreamSynchronize(p->stream));
    color_bytes(p);
    p->sched_dirty = false;
    return BD3MG_OK;
}

template <typename T>
bd3mg_status residual_t(bd3mg_problem p, const T *xin, T *rout)
{
    DevState<T> s = dev_state<T>(p);
    HIP_TRY(launch_H<T>(p->geom, s, xin, (const T *)p->y, rout, p->d_chunks, p->nchunks, p->stream));
    return BD3MG_OK;
}

bd3mg_status residual(bd3mg_problem p, const void *xin, void *rout)
{
    return p->prec == BD3MG_FP64 ? residual_t<double>(p, (const double *)xin, (double *)rout)
                                 : residual_t<float>(p, (const float *)xin, (float *)rout);
}

// f and ||grad f|| at xin with residual rin (whole-volume gradient pass in
// evaluation mode; partial sums reduced in a fixed order on the device).
template <typename T>
bd3mg_status eval_t(bd3mg_problem p, const T *xin, const T *rin, double *f, double *gn)
{
    DevState<T> s = dev_state<T>(p);
    s.x = (T *)xin;
    HIP_TRY(launch_grad<T>(p->geom, p->prm, s, rin, nullptr, p->d_chunks, p->nchunks, GM_EVAL,
                           p->d_partials, p->stream));
    HIP_TRY(launch_sum_eval(p->d_partials, p->geom.ntx * p->geom.nty * p->nchunks, p->d_eval,
                            p->stream));
    double q[NE];
    HIP_TRY(hipMemcpyAsync(q, p->d_eval, sizeof(q), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (f) *f = 0.5 * q[1] + p->prm.eta * q[3] + p->prm.lambda * q[2] + p->prm.kappa * q[4];
    if (gn) *gn = std::sqrt(q[0]);
    return BD3MG_OK;
}

bd3mg_status eval_at(bd3mg_problem p, const void *xin, const void *rin, double *f, double *gn)
{
    return p->prec == BD3MG_FP64
               ? eval_t<double>(p, (const double *)xin, (const double *)rin, f, gn)
               : eval_t<float>(p, (const float *)xin, (const float *)rin, f, gn);
}

bd3mg_status ensure_ready(bd3mg_problem p)
{
    if (!p->psf_set) return fail(BD3MG_ERR_STATE, "the PSF is not set");
    if (!p->data_set) return fail(BD3MG_ERR_STATE, "the data y is not set");
    ST_TRY(build_schedule(p));
    if (!p->x_set) {
        HIP_TRY(hipMemcpyAsync(p->x, p->y, p->N * p->esz, hipMemcpyDeviceToDevice, p->stream));
        ST_TRY(zero_steps(p));
        p->x_set = true;
        p->r_stale = true;
        p->sweeps_done = 0;
    }
    if (!p->gnorm_ref_valid) {
        ST_TRY(ensure_tmp(p, 1));
        ST_TRY(residual(p, p->y, p->tmp[0]));
        ST_TRY(eval_at(p, p->y, p->tmp[0], nullptr, &p->gnorm_ref));
        p->gnorm_ref_valid = true;
    }
    if (p->r_stale) {
        ST_TRY(residual(p, p->x, p->r));
        p->r_stale = false;
    }
    return BD3MG_OK;
}

// Enqueue the four passes of one colour phase over nseg segments.  cb (may be
// null) holds the algorithmic bytes of the four passes for the profile.
template <typename T>
bd3mg_status phase_t(bd3mg_problem p, const Segment *segs, int nseg, const double *cb)
{
    DevState<T> s = dev_state<T>(p);
    const int slots = p->geom.ntx * p->geom.nty;
    ST_TRY(prof_begin(p, BD3MG_K_GRAD, cb ? cb[0] : 0.0));
    HIP_TRY(launch_grad<T>(p->geom, p->prm, s, s.r, nullptr, segs, nseg, GM_BLOCK, p->d_partials,
                           p->stream));
    ST_TRY(prof_end(p));
    ST_TRY(prof_begin(p, BD3MG_K_DIRS, cb ? cb[1] : 0.0));
    HIP_TRY(launch_dirs<T>(p->geom, p->prm, s, segs, nseg, p->d_partials, p->stream));
    ST_TRY(prof_end(p));
    ST_TRY(prof_begin(p, BD3MG_K_SOLVE, cb ? cb[2] : 0.0));
    HIP_TRY(launch_solve(p->prm, segs, nseg, slots, p->d_partials, p->d_u, p->d_info, p->stream));
    ST_TRY(prof_end(p));
    ST_TRY(prof_begin(p, BD3MG_K_UPDATE, cb ? cb[3] : 0.0));
    HIP_TRY(launch_update<T>(p->geom, s, segs, nseg, p->d_u, p->stream));
    ST_TRY(prof_end(p));
    return BD3MG_OK;
}

bd3mg_status phase(bd3mg_problem p, const Segment *segs, int nseg, const double *cb)
{
    return p->prec == BD3MG_FP64 ? phase_t<double>(p, segs, nseg, cb)
                                 : phase_t<float>(p, segs, nseg, cb);
}

bd3mg_status validate_handle(bd3mg_problem p)
{
    if (!p) return fail(BD3MG_ERR_ARG, "null problem handle");
    return BD3MG_OK;
}

}  // namespace

extern "C" {

int bd3mg_version(void) { return (0 << 16) | 1; }

const char *bd3mg_last_error(void) { return g_err.c_str(); }

bd3mg_status bd3mg_psf_gaussian(int nz, int k, const double *sigma, double *table)
{
    if (nz < 1 || k < 1 || (k % 2) == 0) return fail(BD3MG_ERR_ARG, "need nz >= 1 and odd k >= 1");
    if (!sigma || !table) return fail(BD3MG_ERR_ARG, "null array");
    const int r = k / 2;
    for (int z = 0; z < nz; ++z) {
        const double s = sigma[z];
        if (!(s > 0.0) || !std::isfinite(s)) return fail(BD3MG_ERR_ARG, "sigma[%d] must be > 0", z);
        double sum = 0.0;
        double *row = table + (size_t)z * k;
        for (int a = -r; a <= r; ++a) {
            row[a + r] = std::exp(-(double)a * a / (2.0 * s * s));
            sum += row[a + r];
        }
        for (int a = 0; a < k; ++a) row[a] /= sum;
    }
    return BD3MG_OK;
}

bd3mg_status bd3mg_create(int nx, int ny, int nz, int precision, bd3mg_problem *out)
{
    if (!out) return fail(BD3MG_ERR_ARG, "null output handle");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(BD3MG_ERR_ARG, "dimensions must be >= 1");
    if (precision != BD3MG_FP64 && precision != BD3MG_FP32)
        return fail(BD3MG_ERR_ARG, "unknown precision %d", precision);
    bd3mg_problem p = new (std::nothrow) bd3mg_problem_s;
    if (!p) return fail(BD3MG_ERR_NOMEM, "handle");
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->prec = precision;
    p->N = (size_t)nx * ny * nz;
    p->esz = precision == BD3MG_FP64 ? sizeof(double) : sizeof(float);
    p->refresh_every = precision == BD3MG_FP64 ? 0 : 64;
    p->geom.nx = nx;
    p->geom.ny = ny;
    p->geom.nz = nz;
    p->geom.ntx = (nx + TX - 1) / TX;
    p->geom.nty = (ny + TY - 1) / TY;
    auto bail = [&](bd3mg_status st, const char *what) {
        bd3mg_destroy(p);
        return fail(st, "%s", what);
    };
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(BD3MG_ERR_HIP, "stream creation failed");
    if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
        return bail(BD3MG_ERR_HIP, "event creation failed");
    void **vols[] = {&p->x, &p->y, &p->r, &p->g, &p->dpb[0], &p->dpb[1]};
    for (void **v : vols)
        if (hipMalloc(v, p->N * p->esz) != hipSuccess) return bail(BD3MG_ERR_NOMEM, "volume allocation failed");
    // whole-volume chunks
    p->nchunks = (nz + CHUNK - 1) / CHUNK;
    std::vector<Segment> ch;
    for (int z = 0; z < nz; z += CHUNK) ch.push_back(Segment{z, std::min(CHUNK, nz - z), -1, 0});
    if (hipMalloc(&p->d_chunks, ch.size() * sizeof(Segment)) != hipSuccess ||
        hipMalloc(&p->d_eval, NE * sizeof(double)) != hipSuccess)
        return bail(BD3MG_ERR_NOMEM, "tables");
    if (hipMemcpy(p->d_chunks, ch.data(), ch.size() * sizeof(Segment), hipMemcpyHostToDevice) != hipSuccess)
        return bail(BD3MG_ERR_HIP, "chunk upload failed");
    if (ensure_partials(p, (size_t)p->geom.ntx * p->geom.nty * p->nchunks * NE) != BD3MG_OK)
        return bail(BD3MG_ERR_NOMEM, "partials");
    if (zero_steps(p) != BD3MG_OK) return bail(BD3MG_ERR_HIP, "clearing steps failed");
    *out = p;
    return BD3MG_OK;
}

bd3mg_status bd3mg_destroy(bd3mg_problem p)
{
    if (!p) return BD3MG_OK;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    void *bufs[] = {p->x, p->y, p->r, p->g, p->dpb[0], p->dpb[1], p->tmp[0], p->tmp[1], p->tmp[2],
                    p->d_gx, p->d_gy, p->d_gz, p->d_segs, p->d_chunks, p->d_partials, p->d_u,
                    p->d_info, p->d_eval};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (auto &q : p->pending) {
        (void)hipEventDestroy(q.a);
        (void)hipEventDestroy(q.b);
    }
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_psf_separable(bd3mg_problem p, int kx, int ky, int kz, const double *gx,
                                     const double *gy, const double *gz)
{
    ST_TRY(validate_handle(p));
    for (int k : {kx, ky, kz})
        if (k < 1 || (k % 2) == 0 || k > 2 * RMAX + 1)
            return fail(BD3MG_ERR_ARG, "kernel sizes must be odd, 1..%d (got %d)", 2 * RMAX + 1, k);
    if (kz > KZMAX) return fail(BD3MG_ERR_ARG, "kz must be <= %d", KZMAX);
    if (!gx || !gy || !gz) return fail(BD3MG_ERR_ARG, "null table");
    ST_TRY(check_finite(gx, (size_t)p->nz * kx, "gx"));
    ST_TRY(check_finite(gy, (size_t)p->nz * ky, "gy"));
    ST_TRY(check_finite(gz, (size_t)p->nz * kz, "gz"));
    const double *src[3] = {gx, gy, gz};
    const int ks[3] = {kx, ky, kz};
    void **dst[3] = {&p->d_gx, &p->d_gy, &p->d_gz};
    for (int t = 0; t < 3; ++t) {
        const size_t n = (size_t)p->nz * ks[t];
        if (*dst[t]) HIP_TRY(hipFree(*dst[t]));
        *dst[t] = nullptr;
        if (hipMalloc(dst[t], n * p->esz) != hipSuccess) return fail(BD3MG_ERR_NOMEM, "PSF table");
        if (p->prec == BD3MG_FP64) {
            HIP_TRY(hipMemcpy(*dst[t], src[t], n * sizeof(double), hipMemcpyHostToDevice));
        } else {
            std::vector<float> f(src[t], src[t] + n);
            HIP_TRY(hipMemcpy(*dst[t], f.data(), n * sizeof(float), hipMemcpyHostToDevice));
        }
    }
    p->kx = kx;
    p->ky = ky;
    p->kz = kz;
    p->geom.rx = kx / 2;
    p->geom.ry = ky / 2;
    p->geom.rz = kz / 2;
    p->psf_set = true;
    p->r_stale = true;
    p->gnorm_ref_valid = false;
    p->sched_dirty = true;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_psf_gaussian(bd3mg_problem p, int kxy, int kz, const double *sigma_xy,
                                    const double *sigma_z)
{
    ST_TRY(validate_handle(p));
    std::vector<double> txy((size_t)p->nz * std::max(kxy, 1)), tz((size_t)p->nz * std::max(kz, 1));
    ST_TRY(bd3mg_psf_gaussian(p->nz, kxy, sigma_xy, txy.data()));
    ST_TRY(bd3mg_psf_gaussian(p->nz, kz, sigma_z, tz.data()));
    return bd3mg_set_psf_separable(p, kxy, kxy, kz, txy.data(), txy.data(), tz.data());
}

bd3mg_status bd3mg_set_params(bd3mg_problem p, double lambda, double delta, double eta,
                              double kappa, double xmin, double xmax)
{
    ST_TRY(validate_handle(p));
    const double v[6] = {lambda, delta, eta, kappa, xmin, xmax};
    ST_TRY(check_finite(v, 6, "parameter"));
    if (!(delta > 0.0)) return fail(BD3MG_ERR_ARG, "delta must be > 0");
    if (lambda < 0.0 || eta < 0.0 || kappa < 0.0)
        return fail(BD3MG_ERR_ARG, "lambda, eta and kappa must be >= 0");
    if (xmin > xmax) return fail(BD3MG_ERR_ARG, "xmin > xmax");
    const bool kappa_changed = (kappa > 0.0) != (p->prm.kappa > 0.0);
    p->prm = Params{lambda, delta, eta, kappa, xmin, xmax};
    p->gnorm_ref_valid = false;
    if (kappa_changed) p->sched_dirty = true;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_data(bd3mg_problem p, const void *y, int on_device)
{
    ST_TRY(validate_handle(p));
    if (!y) return fail(BD3MG_ERR_ARG, "null data");
    ST_TRY(upload(p, p->y, y, on_device));
    p->data_set = true;
    p->r_stale = true;
    p->gnorm_ref_valid = false;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_blocks(bd3mg_problem p, int nblocks, const int *nslices, int schedule)
{
    ST_TRY(validate_handle(p));
    if (nblocks < 1 || !nslices) return fail(BD3MG_ERR_ARG, "need nblocks >= 1 and slice counts");
    if (schedule != BD3MG_SCHED_COLORED && schedule != BD3MG_SCHED_SEQUENTIAL)
        return fail(BD3MG_ERR_ARG, "unknown schedule %d", schedule);
    long sum = 0;
    for (int b = 0; b < nblocks; ++b) {
        if (nslices[b] < 1) return fail(BD3MG_ERR_ARG, "block %d has %d slices", b, nslices[b]);
        sum += nslices[b];
    }
    if (sum != p->nz) return fail(BD3MG_ERR_ARG, "slice counts sum to %ld, not nz = %d", sum, p->nz);
    p->nsl.assign(nslices, nslices + nblocks);
    p->z0.resize(nblocks);
    int z = 0;
    for (int b = 0; b < nblocks; ++b) {
        p->z0[b] = z;
        z += nslices[b];
    }
    p->schedule = schedule;
    p->blocks_set = true;
    p->sched_dirty = true;
    p->sweeps_done = 0;
    ST_TRY(zero_steps(p));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return BD3MG_OK;
}

bd3mg_status bd3mg_get_schedule(bd3mg_problem p, int *ncolors, int *order, int *color)
{
    ST_TRY(validate_handle(p));
    ST_TRY(build_schedule(p));
    if (ncolors) *ncolors = p->ncolors;
    if (order) std::copy(p->order.begin(), p->order.end(), order);
    if (color) std::copy(p->color.begin(), p->color.end(), color);
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_x0(bd3mg_problem p, const void *x0, int on_device)
{
    ST_TRY(validate_handle(p));
    if (x0) {
        ST_TRY(upload(p, p->x, x0, on_device));
    } else {
        if (!p->data_set) return fail(BD3MG_ERR_STATE, "x0 = y needs the data");
        HIP_TRY(hipMemcpyAsync(p->x, p->y, p->N * p->esz, hipMemcpyDeviceToDevice, p->stream));
    }
    ST_TRY(zero_steps(p));
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->x_set = true;
    p->r_stale = true;
    p->sweeps_done = 0;
    return BD3MG_OK;
}

bd3mg_status bd3mg_run(bd3mg_problem p, int max_sweeps, double grad_rtol, int check_every,
                       bd3mg_result *res)
{
    ST_TRY(validate_handle(p));
    if (max_sweeps < 0) return fail(BD3MG_ERR_ARG, "max_sweeps < 0");
    if (check_every < 0) return fail(BD3MG_ERR_ARG, "check_every < 0");
    const bool checking = grad_rtol > 0.0 || check_every > 0;
    if (grad_rtol > 0.0 && check_every == 0) check_every = max_sweeps > 0 ? max_sweeps : 1;
    ST_TRY(ensure_ready(p));
    const double vol = (double)p->N * p->esz;
    HIP_TRY(hipEventRecord(p->ev0, p->stream));
    int done = 0;
    bool conv = false;
    double gn = NAN, f = NAN;
    for (int s = 0; s < max_sweeps; ++s) {
        for (int c = 0; c < p->ncolors; ++c)
            ST_TRY(phase(p, p->d_segs + p->col_off[c], p->col_cnt[c], &p->color_bytes[(size_t)c * 4]));
        p->cur ^= 1;
        ++done;
        ++p->sweeps_done;
        if (p->refresh_every > 0 && (p->sweeps_done % p->refresh_every) == 0) {
            ST_TRY(prof_begin(p, BD3MG_K_EVAL, 3.0 * vol));
            ST_TRY(residual(p, p->x, p->r));
            ST_TRY(prof_end(p));
        }
        const bool last = (s == max_sweeps - 1);
        if (checking && ((done % check_every) == 0 || last)) {
            ST_TRY(prof_begin(p, BD3MG_K_EVAL, 2.0 * vol));
            ST_TRY(eval_at(p, p->x, p->r, &f, &gn));
            ST_TRY(prof_end(p));
            if (grad_rtol > 0.0 && gn <= grad_rtol * p->gnorm_ref) {
                conv = true;
                break;
            }
        }
        if (p->pending.size() > 4096) ST_TRY(prof_collect(p));
    }
    HIP_TRY(hipEventRecord(p->ev1, p->stream));
    HIP_TRY(hipEventSynchronize(p->ev1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    ST_TRY(prof_collect(p));
    if (res) {
        res->sweeps = done;
        res->converged = conv ? 1 : 0;
        res->f = f;
        res->grad_norm = gn;
        res->grad_norm_ref = p->gnorm_ref;
        res->seconds = ms * 1e-3;
    }
    if (grad_rtol > 0.0 && !conv)
        return fail(BD3MG_ERR_NOT_CONVERGED, "||grad f|| / ||grad f(y)|| = %.3e after %d sweeps",
                    gn / p->gnorm_ref, done);
    return BD3MG_OK;
}

bd3mg_status bd3mg_get_x(bd3mg_problem p, void *x, int on_device)
{
    ST_TRY(validate_handle(p));
    if (!x) return fail(BD3MG_ERR_ARG, "null output");
    if (!p->x_set) return fail(BD3MG_ERR_STATE, "no iterate yet");
    return download(p, x, p->x, on_device);
}

bd3mg_status bd3mg_get_dprev(bd3mg_problem p, void *d, int on_device)
{
    ST_TRY(validate_handle(p));
    if (!d) return fail(BD3MG_ERR_ARG, "null output");
    return download(p, d, p->dpb[p->cur], on_device);
}

bd3mg_status bd3mg_get_state(bd3mg_problem p, void *x, void *dprev, void *r, long long *sweeps,
                             int on_device)
{
    ST_TRY(validate_handle(p));
    if (!p->x_set) return fail(BD3MG_ERR_STATE, "no iterate yet");
    if (r && p->r_stale) ST_TRY(ensure_ready(p));
    if (x) ST_TRY(download(p, x, p->x, on_device));
    if (dprev) ST_TRY(download(p, dprev, p->dpb[p->cur], on_device));
    if (r) ST_TRY(download(p, r, p->r, on_device));
    if (sweeps) *sweeps = p->sweeps_done;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_state(bd3mg_problem p, const void *x, const void *dprev, const void *r,
                             long long sweeps, int on_device)
{
    ST_TRY(validate_handle(p));
    if (!x || !dprev) return fail(BD3MG_ERR_ARG, "null state");
    if (sweeps < 0) return fail(BD3MG_ERR_ARG, "sweeps < 0");
    ST_TRY(upload(p, p->x, x, on_device));
    ST_TRY(upload(p, p->dpb[p->cur], dprev, on_device));
    p->x_set = true;
    if (r) {
        ST_TRY(upload(p, p->r, r, on_device));
        p->r_stale = false;
    } else {
        p->r_stale = true;
    }
    p->sweeps_done = sweeps;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_option(bd3mg_problem p, int option, long long value)
{
    ST_TRY(validate_handle(p));
    switch (option) {
    case BD3MG_OPT_REFRESH_EVERY:
        if (value < 0) return fail(BD3MG_ERR_ARG, "refresh interval < 0");
        p->refresh_every = value;
        return BD3MG_OK;
    case BD3MG_OPT_PROFILE:
        ST_TRY(prof_collect(p));
        p->profile = value != 0;
        return BD3MG_OK;
    default:
        return fail(BD3MG_ERR_ARG, "unknown option %d", option);
    }
}

bd3mg_status bd3mg_get_profile(bd3mg_problem p, long long *launches, double *ms, double *bytes,
                               int reset)
{
    ST_TRY(validate_handle(p));
    ST_TRY(prof_collect(p));
    for (int k = 0; k < BD3MG_K_COUNT; ++k) {
        if (launches) launches[k] = p->prof_launches[k];
        if (ms) ms[k] = p->prof_ms[k];
        if (bytes) bytes[k] = p->prof_bytes[k];
        if (reset) {
            p->prof_launches[k] = 0;
            p->prof_ms[k] = 0.0;
            p->prof_bytes[k] = 0.0;
        }
    }
    return BD3MG_OK;
}

bd3mg_status bd3mg_eval(bd3mg_problem p, double *f, double *grad_norm)
{
    ST_TRY(validate_handle(p));
    ST_TRY(ensure_ready(p));
    ST_TRY(residual(p, p->x, p->r));
    return eval_at(p, p->x, p->r, f, grad_norm);
}

bd3mg_status bd3mg_apply(bd3mg_problem p, int op, const void *in, void *out, int on_device)
{
    ST_TRY(validate_handle(p));
    if (!in || !out) return fail(BD3MG_ERR_ARG, "null buffer");
    if (op != BD3MG_OP_H && op != BD3MG_OP_HT && op != BD3MG_OP_GRAD)
        return fail(BD3MG_ERR_ARG, "unknown operator %d", op);
    if (!p->psf_set) return fail(BD3MG_ERR_STATE, "the PSF is not set");
    if (op == BD3MG_OP_GRAD && !p->data_set) return fail(BD3MG_ERR_STATE, "the data y is not set");
    ST_TRY(ensure_tmp(p, 3));
    ST_TRY(upload(p, p->tmp[0], in, on_device));
    if (p->prec == BD3MG_FP64) {
        DevState<double> s = dev_state<double>(p);
        double *ti = (double *)p->tmp[0], *to = (double *)p->tmp[1], *tr = (double *)p->tmp[2];
        if (op == BD3MG_OP_H) {
            HIP_TRY(launch_H<double>(p->geom, s, ti, nullptr, to, p->d_chunks, p->nchunks, p->stream));
        } else if (op == BD3MG_OP_HT) {
            HIP_TRY(launch_grad<double>(p->geom, p->prm, s, ti, to, p->d_chunks, p->nchunks, GM_HT,
                                        nullptr, p->stream));
        } else {
            HIP_TRY(launch_H<double>(p->geom, s, ti, (const double *)p->y, tr, p->d_chunks, p->nchunks,
                                     p->stream));
            s.x = ti;
            HIP_TRY(launch_grad<double>(p->geom, p->prm, s, tr, to, p->d_chunks, p->nchunks, GM_GRAD,
                                        nullptr, p->stream));
        }
    } else {
        DevState<float> s = dev_state<float>(p);
        float *ti = (float *)p->tmp[0], *to = (float *)p->tmp[1], *tr = (float *)p->tmp[2];
        if (op == BD3MG_OP_H) {
            HIP_TRY(launch_H<float>(p->geom, s, ti, nullptr, to, p->d_chunks, p->nchunks, p->stream));
        } else if (op == BD3MG_OP_HT) {
            HIP_TRY(launch_grad<float>(p->geom, p->prm, s, ti, to, p->d_chunks, p->nchunks, GM_HT,
                                       nullptr, p->stream));
        } else {
            HIP_TRY(launch_H<float>(p->geom, s, ti, (const float *)p->y, tr, p->d_chunks, p->nchunks,
                                    p->stream));
            s.x = ti;
            HIP_TRY(launch_grad<float>(p->geom, p->prm, s, tr, to, p->d_chunks, p->nchunks, GM_GRAD,
                                       nullptr, p->stream));
        }
    }
    return download(p, out, p->tmp[1], on_device);
}

bd3mg_status bd3mg_block_step(bd3mg_problem p, int block, double *info)
{
    ST_TRY(validate_handle(p));
    ST_TRY(ensure_ready(p));
    const int nb = (int)p->nsl.size();
    if (block < 0 || block >= nb) return fail(BD3MG_ERR_ARG, "block %d out of range", block);
    const int segi = p->col_off.empty() ? 0 : (int)(p->order.size()) + block;
    ST_TRY(phase(p, p->d_segs + segi, 1, nullptr));
    // keep every block's step in one buffer: copy this block's new step back
    const size_t off = (size_t)p->z0[block] * p->nx * p->ny * p->esz;
    const size_t len = (size_t)p->nsl[block] * p->nx * p->ny * p->esz;
    HIP_TRY(hipMemcpyAsync((char *)p->dpb[p->cur] + off, (char *)p->dpb[p->cur ^ 1] + off, len,
                           hipMemcpyDeviceToDevice, p->stream));
    if (info) {
        HIP_TRY(hipMemcpyAsync(info, p->d_info + 8 * block, 8 * sizeof(double), hipMemcpyDeviceToHost,
                               p->stream));
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    return BD3MG_OK;
}

bd3mg_status bd3mg_probe_copy(size_t bytes, int iters, double *gbps, double *ms)
{
    if (bytes < (1u << 20) || iters < 1) return fail(BD3MG_ERR_ARG, "need bytes >= 1 MiB and iters >= 1");
    const size_t n16 = bytes / 16;
    void *a = nullptr, *b = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bd3mg_status rc = BD3MG_OK;
    float best = 0.f;
    if (hipMalloc(&a, n16 * 16) != hipSuccess || hipMalloc(&b, n16 * 16) != hipSuccess) {
        rc = fail(BD3MG_ERR_NOMEM, "probe buffers of %zu bytes", n16 * 16);
    } else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = fail(BD3MG_ERR_HIP, "probe stream or events");
    } else if (hipMemsetAsync(a, 0, n16 * 16, st) != hipSuccess) {
        rc = fail(BD3MG_ERR_HIP, "probe memset");
    } else {
        for (int it = 0; it <= iters && rc == BD3MG_OK; ++it) {  // first launch warms up
            float t = 0.f;
            if (hipEventRecord(e0, st) != hipSuccess || launch_copy(a, b, n16, st) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess)
                rc = fail(BD3MG_ERR_HIP, "probe launch");
            else if (it > 0 && (best == 0.f || t < best))
                best = t;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (rc != BD3MG_OK) return rc;
    if (ms) *ms = best;
    if (gbps) *gbps = 2.0 * n16 * 16 / (best * 1e-3) / 1e9;
    return BD3MG_OK;
}

}  // extern "C"
