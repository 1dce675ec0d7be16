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
#include <utility>
#include <vector>

#include "../../include/bd3mg.h"
#include "bd3mg_internal.h"

using namespace bd3mg;

namespace bd3mg {

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

}  // namespace bd3mg

struct bd3mg_problem_s {
    int nx = 0, ny = 0, nz = 0, prec = 0;
    size_t N = 0, esz = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;  // created by bd3mg_create (else the caller's)
    int device = 0;           // HIP device the problem lives on
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    Geom geom{};
    int ntiles = 0;
    Params prm{0.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, M_BD3MG, 0.0, 0};
    int n_inner = 0;         // Async-MM: inner iterations at most
    double tol_inner = 0.0;  // Async-MM: relative residual of the inner solve (0: n_inner iterations)
    double lip_given = 0.0;  // L of the metric L Id as given (<= 0: the Lipschitz bound)

    // PSF
    bool psf_set = false;
    int kx = 0, ky = 0, kz = 0;
    void *d_gx = nullptr, *d_gy = nullptr, *d_gz = nullptr;
    std::vector<double> hgx, hgy, hgz;  // the tables as given (for the Lipschitz bound)
    // general per-depth kernels: then the maintained vector q holds r = Hx - y
    bool dense = false;
    void *d_pk = nullptr;    // [nz][kz][2R+1][2R+1], storage type
    void *d_ones = nullptr;  // [nz] ones: the z table of the gradient pass in the dense mode
    void *d_hts = nullptr;   // source shares of H^T r of a launch group (dense mode)
    size_t hts_alloc = 0;
    std::vector<double> hpk;  // [nz][kz][ky][kx] as given

    // volumes (storage type); q is the in-slice adjoint-blurred residual
    void *x = nullptr, *y = nullptr, *q = nullptr, *g = nullptr, *dpb[2] = {nullptr, nullptr};
    void *tmp[4] = {nullptr, nullptr, nullptr, nullptr};  // tmp[3]: H^T r of the dense mode
    // guard of the round schedule: f checked every round_guard sweeps, the last
    // accepted state (x, previous steps, q) kept in gsave
    long long round_guard = 0;
    void *gsave[3] = {nullptr, nullptr, nullptr};
    int guard_trips = 0;  // restores of the last run
    int cur = 0;  // dpb[cur] holds every block's last step
    bool data_set = false, x_set = false, q_stale = true;

    // blocks, schedule and the work-item lists of every launch group
    bool blocks_set = false, sched_dirty = true;
    int schedule = BD3MG_SCHED_COLORED;
    std::vector<int> nsl, z0, order, color;
    int ncolors = 0;
    struct Group {
        int g_off, g_cnt, d_off, d_cnt, u_off, u_cnt, br_off, br_cnt;
        int du_off, du_cnt;  // direction units: one or two consecutive slices of a block
        double bytes[4];  // algorithmic bytes of the gradient, direction, solve and update passes
        bool round;       // update pass over every slice with per-slice block coefficients
        int dbase;        // colour groups: first direction item among all colour groups' items
        double bytes_one; // direction pass blurring d1 only (H dp read)
        double bytes_hdw; // update pass: the stores of every pair's H d'
    };
    std::vector<Group> groups;  // ncolors colour groups, then one group per block
    Item *d_items = nullptr;
    size_t items_alloc = 0;
    BlockRange *d_br = nullptr;
    size_t br_alloc = 0;
    Item *d_vol = nullptr;  // every slice of the volume, for whole-volume passes
    int *d_sblk = nullptr;  // block of every slice
    int2 *d_pairs = nullptr;  // (direction slot, block) sources of the update items
    size_t pairs_alloc = 0;
    Item *d_units = nullptr;  // direction workgroups: slice, block, first direction item, slice count
    size_t units_alloc = 0;
    int dirs_slices = 0;      // slices per direction workgroup (0: by group size)
    void *d_hd = nullptr;     // H d1 then H d2 of a launch group's direction items
    size_t hd_alloc = 0, hd_slots = 0;
    // H dp of every colour group's direction items, the update pass's H d'
    // kept for the block's next visit: two buffers of hdp_slots slots, the
    // one read selected by the parity of cur (as dpb)
    void *d_hdp = nullptr;
    size_t hdp_alloc = 0, hdp_slots = 0;
    long long hdp_every = 64;  // sweeps 0, n, 2n, ... (counted from x^0) blur both directions (0: H dp never kept)
    int stream_stores = -1;    // BD3MG_OPT_STREAM_STORES: -1 by volume size, 0 off, 1 on
    bool hdp_valid = false;    // the buffer cur selects holds H dp of every block
    int maxg = 1, maxd = 1;   // most gradient and direction items of a launch group

    // reductions
    double *d_pg = nullptr, *d_pd = nullptr, *d_pe = nullptr, *d_pr = nullptr;
    size_t pg_cap = 0, pd_cap = 0;
    double *d_u = nullptr, *d_info = nullptr, *d_sum = nullptr;
    // device stop test: {int stop, int stop_sweep, double gnorm}
    struct Ctl {
        int stop;
        int stop_sweep;
        double gnorm;
    };
    Ctl *d_ctl = nullptr;
    int nblocks_alloc = 0;

    // Async-MM's inner solve: r, p, v, A p, XY^T (H p) volumes, partial sums
    // and per-block scalars
    void *mmv[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double *d_pma = nullptr, *d_prr = nullptr, *d_cgs = nullptr, *d_u01 = nullptr, *d_u10 = nullptr;
    size_t mm_slots = 0;
    int mm_blocks = 0;

    double gnorm_ref = 0.0;
    bool gnorm_ref_valid = false;

    long long sweeps_done = 0;  // sweeps since x^0 (drives the refresh of q)
    long long refresh_every = 0;

    // profiling: start and end events of the launches not yet folded into
    // the totals (a single-kernel pass: the kernel's own start and end
    // timestamps; a pass of several kernels: events recorded around them)
    bool profile = false;
    struct Pending {
        int kind;
        double bytes;
        hipEvent_t a, b;
        bool own;  // a, b are the kernel's own start and stop events
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    long long prof_launches[BD3MG_K_COUNT] = {0, 0, 0, 0, 0};
    double prof_ms[BD3MG_K_COUNT] = {0, 0, 0, 0, 0};
    double prof_bytes[BD3MG_K_COUNT] = {0, 0, 0, 0, 0};
};

namespace {

// Non-temporal stores of the gradient and update passes' volume outputs
// (BD3MG_OPT_STREAM_STORES): by default when one volume of the problem holds
// at least 64 MiB, where a colour's passes move several times the GPU's L2
// and Infinity Cache and kept lines are evicted before the next pass reads
// them (measured in FP32: 512 x 512 x 128 sweeps 1.078 -> 1.040 ms; on
// 256 x 256 x 64 the hint would cost 3 %).
bool stream_stores(bd3mg_problem p)
{
    if (p->stream_stores >= 0) return p->stream_stores != 0;
    return (double)p->N * p->esz >= 64.0 * 1024 * 1024;
}

template <typename T>
DevState<T> dev_state(bd3mg_problem p)
{
    DevState<T> s;
    s.x = (T *)p->x;
    s.y = (T *)p->y;
    s.q = (T *)p->q;
    s.g = (T *)p->g;
    s.dp[0] = (T *)p->dpb[p->cur];
    s.dp[1] = (T *)p->dpb[p->cur ^ 1];
    s.gx = (const T *)p->d_gx;
    s.gy = (const T *)p->d_gy;
    s.gz = (const T *)p->d_gz;
    s.sblk = p->d_sblk;
    s.hd[0] = (T *)p->d_hd;
    s.hd[1] = s.hd[0] ? s.hd[0] + p->hd_slots * p->nx * p->ny : nullptr;
    s.hdw = nullptr;
    s.stop = nullptr;
    s.nt = stream_stores(p) ? 1 : 0;
    return s;
}

// Gradient pass of the dense mode: H^T r on the items' slices into tmp[3] by
// the general-kernel adjoint, then the gradient kernel with a one-tap z table
// reading it (the rest of grad f and the partial sums as in the separable
// mode).
// Source shares of the adjoint for n output slices: enough workgroups to
// fill the GPU when a group has few slices (at least two sources a share).
int dense_split(bd3mg_problem p, int n, int ty)
{
    const int wgs = n * tiles_of(p->geom, ty);
    const int ns = (1024 + wgs - 1) / std::max(wgs, 1);
    return std::max(1, std::min(ns, (p->kz + 1) / 2));
}

template <typename T>
hipError_t dense_grad(bd3mg_problem p, const DevState<T> &s, const T *r, const T *x, T *out,
                      const Item *items, int n, int mode, double *partials, bool split = false,
                      T *ht_buf = nullptr)
{
    const int ns = split ? dense_split(p, n, p->geom.ty_dirs) : 1;
    // shares of H^T r stay in d_hts and the gradient kernel adds them; one
    // share goes to ht_buf (a volume; the problem's scratch volume when null)
    T *ht = ns > 1 ? nullptr : (ht_buf ? ht_buf : (T *)p->tmp[3]);
    hipError_t e = launch_dense<T>(p->geom, p->prm, s, (const T *)p->d_pk, r, nullptr, ht, items, n, DM_HT,
                                   nullptr, p->stream, ns, (T *)p->d_hts);
    if (e != hipSuccess) return e;
    Geom g1 = p->geom;
    g1.rz = 0;
    DevState<T> s1 = s;
    s1.gz = (const T *)p->d_ones;
    return launch_grad<T>(g1, p->prm, s1, ns > 1 ? (const T *)p->d_hts : ht, x, out, items, n, mode, partials,
                          p->stream, ns > 1 ? ns : 0);
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

// Start of a profiled pass (no-op unless profiling).  A pass of one kernel
// hands its events to the launcher (hipExtLaunchKernelGGL timestamps the
// kernel itself); a pass of several kernels records events around them.
bd3mg_status prof_begin(bd3mg_problem p, int kind, double bytes, bool one_kernel = true)
{
    if (!p->profile) return BD3MG_OK;
    bd3mg_problem_s::Pending q{kind, bytes, pool_event(p), pool_event(p), one_kernel};
    if (!q.a || !q.b) return fail(BD3MG_ERR_HIP, "event creation failed");
    if (one_kernel)
        g_launch_events = LaunchEvents{q.a, q.b};
    else
        HIP_TRY(hipEventRecord(q.a, p->stream));
    p->pending.push_back(q);
    return BD3MG_OK;
}

bd3mg_status prof_end(bd3mg_problem p)
{
    if (!p->profile) return BD3MG_OK;
    if (p->pending.back().own)
        g_launch_events = LaunchEvents{};
    else
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

bd3mg_status realloc_dev(void **ptr, size_t *cap, size_t bytes, const char *what)
{
    if (bytes <= *cap && *ptr) return BD3MG_OK;
    if (*ptr) HIP_TRY(hipFree(*ptr));
    *ptr = nullptr;
    *cap = 0;
    if (hipMalloc(ptr, bytes) != hipSuccess) return fail(BD3MG_ERR_NOMEM, "%s (%zu bytes)", what, bytes);
    *cap = bytes;
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
    p->hdp_valid = false;
    return BD3MG_OK;
}

// Whether the criterion couples neighbouring slices outside H: the z
// penalty, or the total variation taken along z.
static bool z_coupled(bd3mg_problem p) { return p->prm.kappa > 0.0 || p->prm.tv3d; }

// Greedy colouring in z order: block b takes the smallest colour none of whose
// earlier members is closer than min_gap slices.  Same-colour blocks then read
// and write disjoint data (the residual on S +- r_z, the iterate on S +- 1 when
// kappa > 0 or the TV is taken along z), so updating them together equals
// updating them in sequence.
void color_blocks(bd3mg_problem p)
{
    const int nb = (int)p->nsl.size();
    p->color.assign(nb, 0);
    p->order.clear();
    if (p->schedule == BD3MG_SCHED_SEQUENTIAL) {
        for (int b = 0; b < nb; ++b) p->color[b] = b;
        p->ncolors = nb;
    } else if (p->schedule == BD3MG_SCHED_ROUND) {
        p->ncolors = 1;  // every block in one round, all from the same snapshot
    } else {
        const int rz = p->kz / 2;
        const int min_gap = std::max(2 * rz, z_coupled(p) ? 1 : 0);
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

// Work items of a launch group (a set of blocks updated together):
//   gradient pass: the blocks' own slices S;
//   direction pass: S +- r_z (and slice z0 - 1 when kappa > 0 or the TV is
//   taken along z, for VZ);
//   update pass: S +- r_z (a round: every slice of the volume once),
// all clipped to the volume, block by block in z order.  Each update item
// lists its sources: the (direction slot, block) pairs whose stored H d1,
// H d2 on the item's slice make up H d' there.
void group_items(bd3mg_problem p, const std::vector<int> &blocks, std::vector<Item> &gi,
                 std::vector<Item> &di, std::vector<Item> &ui, std::vector<int2> &pairs,
                 std::vector<Item> &units, std::vector<BlockRange> &br, bd3mg_problem_s::Group &grp,
                 bool round = false)
{
    const int rz = p->kz / 2;
    const int rd = std::max(rz, z_coupled(p) ? 1 : 0);
    grp.g_off = (int)gi.size();
    grp.d_off = (int)di.size();
    grp.dbase = (int)di.size();
    grp.u_off = (int)ui.size();
    grp.br_off = (int)br.size();
    grp.du_off = (int)units.size();
    std::vector<char> halo(p->nz, 0);
    std::vector<int> dfirst, dlo, dend;  // per block of the group: direction slots, first slice
    double sl = 0.0, np = 0.0;
    for (int b : blocks) {
        const int z0 = p->z0[b], n = p->nsl[b];
        BlockRange r{b, (int)gi.size() - grp.g_off, 0, (int)di.size() - grp.d_off, 0};
        // gradient items carry the block's first gradient item (in the group)
        // and its item count: the slots of the block's partial sums
        for (int k = z0; k < z0 + n; ++k) gi.push_back(Item{k, b, z0, n, r.g0, n});
        const int lo = std::max(0, z0 - rd);
        dfirst.push_back(r.d0);
        dlo.push_back(lo);
        for (int k = lo; k < std::min(p->nz, z0 + n + rz); ++k) di.push_back(Item{k, b, z0, n, 0, 0});
        dend.push_back((int)di.size() - grp.d_off);
        if (!round)
            for (int k = std::max(0, z0 - rz); k < std::min(p->nz, z0 + n + rz); ++k) {
                ui.push_back(Item{k, b, z0, n, (int)pairs.size(), 1, r.d0 + k - lo, b});
                pairs.push_back(int2{r.d0 + k - lo, b});
                halo[k] = 1;
            }
        r.gn = (int)gi.size() - grp.g_off - r.g0;
        r.dn = (int)di.size() - grp.d_off - r.d0;
        br.push_back(r);
        sl += n;
    }
    if (round) {
        // one update item per slice of the volume, with a source pair for
        // every block whose S +- r_z holds the slice; x and dp are updated
        // with the coefficients of the slice's own block
        for (int k = 0; k < p->nz; ++k) {
            int b = 0;
            while (p->z0[b] + p->nsl[b] <= k) ++b;
            const int h0 = (int)pairs.size();
            for (size_t t = 0; t < blocks.size(); ++t) {
                const int c = blocks[t], z0 = p->z0[c], z1 = z0 + p->nsl[c];
                if (k >= z0 - rz && k < z1 + rz) pairs.push_back(int2{dfirst[t] + k - dlo[t], c});
            }
            const int2 first = (int)pairs.size() > h0 ? pairs[h0] : int2{0, 0};
            ui.push_back(Item{k, b, p->z0[b], p->nsl[b], h0, (int)pairs.size() - h0, first.x, first.y});
            halo[k] = 1;
        }
    }
    for (int t = grp.u_off; t < (int)ui.size(); ++t) np += ui[t].hn;
    // A direction workgroup takes two consecutive slices of a block (sharing
    // the reads of their common source slices) when the group has enough
    // direction outputs to keep every compute unit busy with half as many
    // workgroups (at least 2^20 voxels), else one.
    const int ndir = (int)di.size() - grp.d_off;
    const int per = p->dirs_slices > 0 ? p->dirs_slices
                                       : ((double)ndir * p->nx * p->ny >= (double)(1 << 20) ? 2 : 1);
    for (size_t t = 0; t < dfirst.size(); ++t)
        for (int i = dfirst[t]; i < dend[t]; i += per) {
            const Item &d = di[grp.d_off + i];
            units.push_back(Item{d.k, d.block, d.z0, d.n, i, std::min(per, dend[t] - i), 0, 0});
        }
    // the two-slice units first: when the grid takes more than one round of
    // residency, the workgroups that start late are those of the one-slice
    // units, about half the work (each unit's partial sums go to its own
    // items' slots, so the order changes no result)
    std::stable_partition(units.begin() + grp.du_off, units.end(), [](const Item &u) { return u.hn > 1; });
    grp.round = round;
    grp.du_cnt = (int)units.size() - grp.du_off;
    grp.g_cnt = (int)gi.size() - grp.g_off;
    grp.d_cnt = (int)di.size() - grp.d_off;
    grp.u_cnt = (int)ui.size() - grp.u_off;
    grp.br_cnt = (int)br.size() - grp.br_off;
    double h = 0.0;
    for (char c : halo) h += c;
    // Algorithmic bytes (every element a pass must read or write counted once):
    // gradient pass reads q on S +- r_z and x, dp on S and writes g on S;
    // direction pass reads g and dp on S and writes H d1, H d2 of its items;
    // solve reads the partial sums; update pass reads H d1, H d2 of its source
    // pairs, g, dp, x on S and q on S +- r_z, writes x, dp on S and q on S +- r_z.
    const double A = (double)p->nx * p->ny * p->esz;
    // (dense mode: the gradient pass also writes and reads H^T r on S)
    grp.bytes[0] = A * (h + (p->dense ? 5.0 : 3.0) * sl);
    grp.bytes[1] = A * (2.0 * sl + 2.0 * grp.d_cnt);
    grp.bytes[2] = (double)(grp.g_cnt * NQG + grp.d_cnt * NQD) * p->ntiles * sizeof(double);
    grp.bytes[3] = A * (2.0 * np + 5.0 * sl + 2.0 * h);
    // reading H dp instead of dp and blurring d1 only: g on S and H dp of
    // the items read, H d1 written; the update pass then also writes H d'
    grp.bytes_one = A * (sl + 2.0 * grp.d_cnt);
    grp.bytes_hdw = A * np;
}

// Buffers of Async-MM's inner solve for launch groups of at most maxg
// gradient items (five volumes, two partial-sum arrays, block scalars, and
// the constant coefficient pairs (0, 1) and (1, 0) of every block).
bd3mg_status ensure_mm(bd3mg_problem p, int maxg)
{
    for (void *&v : p->mmv)
        if (!v && hipMalloc(&v, p->N * p->esz) != hipSuccess) return fail(BD3MG_ERR_NOMEM, "Async-MM volumes");
    const size_t slots = (size_t)maxg * p->ntiles;
    if (slots > p->mm_slots) {
        if (p->d_pma) HIP_TRY(hipFree(p->d_pma));
        if (p->d_prr) HIP_TRY(hipFree(p->d_prr));
        p->d_pma = p->d_prr = nullptr;
        p->mm_slots = 0;
        if (hipMalloc(&p->d_pma, slots * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->d_prr, slots * sizeof(double)) != hipSuccess)
            return fail(BD3MG_ERR_NOMEM, "Async-MM partial sums");
        p->mm_slots = slots;
    }
    const int nb = (int)p->nsl.size();
    if (nb > p->mm_blocks) {
        for (double **d : {&p->d_cgs, &p->d_u01, &p->d_u10}) {
            if (*d) HIP_TRY(hipFree(*d));
            *d = nullptr;
        }
        p->mm_blocks = 0;
        if (hipMalloc(&p->d_cgs, (size_t)CG_STRIDE * nb * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->d_u01, 2 * (size_t)nb * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->d_u10, 2 * (size_t)nb * sizeof(double)) != hipSuccess)
            return fail(BD3MG_ERR_NOMEM, "Async-MM block scalars");
        p->mm_blocks = nb;
    }
    std::vector<double> u01(2 * nb), u10(2 * nb);
    for (int b = 0; b < nb; ++b) {
        u01[2 * b] = 0.0;
        u01[2 * b + 1] = 1.0;
        u10[2 * b] = 1.0;
        u10[2 * b + 1] = 0.0;
    }
    HIP_TRY(hipMemcpy(p->d_u01, u01.data(), u01.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->d_u10, u10.data(), u10.size() * sizeof(double), hipMemcpyHostToDevice));
    return BD3MG_OK;
}

bd3mg_status build_schedule(bd3mg_problem p)
{
    if (!p->sched_dirty) return BD3MG_OK;
    if (!p->blocks_set) return fail(BD3MG_ERR_STATE, "blocks are not set");
    if (!p->psf_set) return fail(BD3MG_ERR_STATE, "the PSF is not set (the colouring needs r_z)");
    color_blocks(p);
    const int nb = (int)p->nsl.size();
    std::vector<Item> gi, di, ui;
    std::vector<int2> pairs;
    std::vector<Item> units;
    std::vector<BlockRange> br;
    p->groups.assign(p->ncolors + nb, bd3mg_problem_s::Group{});
    for (int c = 0; c < p->ncolors; ++c) {
        std::vector<int> blocks;
        for (int b : p->order)
            if (p->color[b] == c) blocks.push_back(b);
        group_items(p, blocks, gi, di, ui, pairs, units, br, p->groups[c], p->schedule == BD3MG_SCHED_ROUND);
    }
    const size_t ndc = di.size();  // direction items of the colour groups
    for (int b = 0; b < nb; ++b) group_items(p, {b}, gi, di, ui, pairs, units, br, p->groups[p->ncolors + b]);
    // one device array: gradient items, then direction items, then update items
    const int ng = (int)gi.size(), nd = (int)di.size();
    for (auto &grp : p->groups) {
        grp.d_off += ng;
        grp.u_off += ng + nd;
    }
    std::vector<Item> all(gi);
    all.insert(all.end(), di.begin(), di.end());
    all.insert(all.end(), ui.begin(), ui.end());
    ST_TRY(realloc_dev((void **)&p->d_items, &p->items_alloc, all.size() * sizeof(Item), "work items"));
    ST_TRY(realloc_dev((void **)&p->d_br, &p->br_alloc, br.size() * sizeof(BlockRange), "block ranges"));
    HIP_TRY(hipMemcpyAsync(p->d_items, all.data(), all.size() * sizeof(Item), hipMemcpyHostToDevice,
                           p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_br, br.data(), br.size() * sizeof(BlockRange), hipMemcpyHostToDevice,
                           p->stream));
    ST_TRY(realloc_dev((void **)&p->d_pairs, &p->pairs_alloc, pairs.size() * sizeof(int2), "update sources"));
    HIP_TRY(hipMemcpyAsync(p->d_pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice,
                           p->stream));
    ST_TRY(realloc_dev((void **)&p->d_units, &p->units_alloc, units.size() * sizeof(Item), "direction units"));
    HIP_TRY(hipMemcpyAsync(p->d_units, units.data(), units.size() * sizeof(Item), hipMemcpyHostToDevice,
                           p->stream));
    {
        std::vector<int> sblk(p->nz);
        for (int b = 0; b < nb; ++b)
            for (int k = p->z0[b]; k < p->z0[b] + p->nsl[b]; ++k) sblk[k] = b;
        if (!p->d_sblk && hipMalloc(&p->d_sblk, p->nz * sizeof(int)) != hipSuccess)
            return fail(BD3MG_ERR_NOMEM, "slice blocks");
        HIP_TRY(hipMemcpy(p->d_sblk, sblk.data(), p->nz * sizeof(int), hipMemcpyHostToDevice));
    }
    if (nb > p->nblocks_alloc) {
        if (p->d_u) HIP_TRY(hipFree(p->d_u));
        if (p->d_info) HIP_TRY(hipFree(p->d_info));
        p->d_u = p->d_info = nullptr;
        if (hipMalloc(&p->d_u, 2 * nb * sizeof(double)) != hipSuccess ||
            hipMalloc(&p->d_info, 8 * nb * sizeof(double)) != hipSuccess)
            return fail(BD3MG_ERR_NOMEM, "per-block coefficients");
        p->nblocks_alloc = nb;
    }
    int maxg = 1, maxd = 1;
    for (auto &grp : p->groups) {
        maxg = std::max(maxg, grp.g_cnt);
        maxd = std::max(maxd, grp.d_cnt);
    }
    p->maxg = maxg;
    p->maxd = maxd;
    if (p->prm.method == M_MM) ST_TRY(ensure_mm(p, maxg));
    ST_TRY(realloc_dev((void **)&p->d_pg, &p->pg_cap, (size_t)maxg * p->ntiles * NQG * sizeof(double),
                       "gradient partial sums"));
    ST_TRY(realloc_dev((void **)&p->d_pd, &p->pd_cap,
                       (size_t)maxd * tiles_of(p->geom, 16) * NQD * sizeof(double),
                       "direction partial sums"));
    // H d1 and H d2 of the largest group's direction items
    ST_TRY(realloc_dev(&p->d_hd, &p->hd_alloc, 2 * (size_t)maxd * p->nx * p->ny * p->esz,
                       "stored directions H d1, H d2"));
    p->hd_slots = (size_t)maxd;
    p->hdp_slots = ndc;
    p->hdp_valid = false;
    if (p->dense) {
        ST_TRY(ensure_tmp(p, 4));  // H^T r of the gradient pass
        size_t sl = 1;
        // for either tile height (the autotuner may change it after this)
        for (auto &grp : p->groups)
            for (int ty : {16, 32}) sl = std::max(sl, (size_t)dense_split(p, grp.g_cnt, ty) * grp.g_cnt);
        ST_TRY(realloc_dev(&p->d_hts, &p->hts_alloc, sl * p->nx * p->ny * p->esz, "adjoint source shares"));
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->sched_dirty = false;
    return BD3MG_OK;
}

// q = XY^T (H src - y), slice by slice, into qout (skipped once *stop is set).
template <typename T>
bd3mg_status refresh_t(bd3mg_problem p, const T *src, T *qout, const int *stop)
{
    DevState<T> s = dev_state<T>(p);
    s.stop = stop;
    if (p->dense) {
        HIP_TRY(launch_dense<T>(p->geom, p->prm, s, (const T *)p->d_pk, src, s.y, qout, p->d_vol, p->nz, DM_H,
                                nullptr, p->stream));
        return BD3MG_OK;
    }
    HIP_TRY(launch_refresh<T>(p->geom, s, src, qout, p->d_vol, p->nz, p->stream));
    return BD3MG_OK;
}

bd3mg_status refresh(bd3mg_problem p, const void *src, void *qout, const int *stop = nullptr)
{
    return p->prec == BD3MG_FP64 ? refresh_t<double>(p, (const double *)src, (double *)qout, stop)
                                 : refresh_t<float>(p, (const float *)src, (float *)qout, stop);
}

// Enqueue the stop test: evaluation pass of ||grad f|| from q, then k_check
// (threshold thr; thr < 0 only records the norm).  No host synchronisation.
template <typename T>
bd3mg_status check_t(bd3mg_problem p, double thr, int sweep, int *stop)
{
    DevState<T> s = dev_state<T>(p);
    s.stop = stop;
    if (p->dense) {
        HIP_TRY(dense_grad<T>(p, s, s.q, s.x, nullptr, p->d_vol, p->nz, GM_EVAL, p->d_pe));
    } else {
        HIP_TRY(launch_grad<T>(p->geom, p->prm, s, s.q, s.x, nullptr, p->d_vol, p->nz, GM_EVAL, p->d_pe,
                               p->stream));
    }
    HIP_TRY(launch_check(p->d_pe, p->ntiles * p->nz, thr, sweep, &p->d_ctl->stop, &p->d_ctl->stop_sweep,
                         &p->d_ctl->gnorm, p->stream));
    return BD3MG_OK;
}

bd3mg_status check(bd3mg_problem p, double thr, int sweep, int *stop)
{
    return p->prec == BD3MG_FP64 ? check_t<double>(p, thr, sweep, stop) : check_t<float>(p, thr, sweep, stop);
}

// ||grad f(xin)|| from the blurred residual qin, and, when f is wanted, f(xin)
// (which needs the residual itself: one H pass into a volume, hbuf, or the
// problem's scratch volume when null).  Sums are reduced in a fixed order on
// the device.
template <typename T>
bd3mg_status eval_t(bd3mg_problem p, const T *xin, const T *qin, double *f, double *gn, T *hbuf)
{
    DevState<T> s = dev_state<T>(p);
    const int nslot = p->ntiles * p->nz;
    if (p->dense) {
        ST_TRY(ensure_tmp(p, 4));
        HIP_TRY(dense_grad<T>(p, s, qin, xin, nullptr, p->d_vol, p->nz, GM_EVAL, p->d_pe));
    } else {
        HIP_TRY(launch_grad<T>(p->geom, p->prm, s, qin, xin, nullptr, p->d_vol, p->nz, GM_EVAL, p->d_pe,
                               p->stream));
    }
    HIP_TRY(launch_sum(p->d_pe, nslot, NQE, p->d_sum, p->stream));
    if (f) {
        if (!hbuf) {
            ST_TRY(ensure_tmp(p, 1));
            hbuf = (T *)p->tmp[0];
        }
        if (p->dense) {
            HIP_TRY(launch_dense<T>(p->geom, p->prm, s, (const T *)p->d_pk, xin, (const T *)p->y, hbuf,
                                    p->d_vol, p->nz, DM_H, p->d_pr, p->stream));
            HIP_TRY(launch_sum(p->d_pr, tiles_of(p->geom, p->geom.ty_dirs) * p->nz, 1, p->d_sum + NQE,
                               p->stream));
        } else {
            HIP_TRY(launch_H<T>(p->geom, s, xin, (const T *)p->y, hbuf, p->d_vol, p->nz, p->d_pr, p->stream));
            HIP_TRY(launch_sum(p->d_pr, tiles_of(p->geom, p->geom.ty_aux) * p->nz, 1, p->d_sum + NQE,
                               p->stream));
        }
    }
    double q[NQE + 1] = {0, 0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(q, p->d_sum, (f ? NQE + 1 : NQE) * sizeof(double), hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (f) *f = 0.5 * q[NQE] + p->prm.lambda * q[1] + p->prm.eta * q[2] + p->prm.kappa * q[3];
    if (gn) *gn = std::sqrt(q[0]);
    return BD3MG_OK;
}

bd3mg_status eval_at(bd3mg_problem p, const void *xin, const void *qin, double *f, double *gn,
                     void *hbuf = nullptr)
{
    return p->prec == BD3MG_FP64
               ? eval_t<double>(p, (const double *)xin, (const double *)qin, f, gn, (double *)hbuf)
               : eval_t<float>(p, (const float *)xin, (const float *)qin, f, gn, (float *)hbuf);
}

// The method's settings that depend on the PSF, parameters and schedule:
// L of the metric L Id (Async-GD, Async-CG) when not given; Async-MM needs
// the separable PSF and blocks whose S +- r_z are disjoint within a launch
// group (coloured or sequential schedule).
bd3mg_status method_ready(bd3mg_problem p)
{
    if (p->prm.method == M_GD || p->prm.method == M_CG) {
        if (p->lip_given > 0.0) {
            p->prm.lip = p->lip_given;
        } else {
            double L = 0.0;
            ST_TRY(bd3mg_lipschitz_bound(p, &L));
            p->prm.lip = L;
        }
    }
    if (p->prm.method == M_MM) {
        if (p->dense) return fail(BD3MG_ERR_STATE, "Async-MM runs with the separable PSF");
        if (p->schedule == BD3MG_SCHED_ROUND)
            return fail(BD3MG_ERR_STATE, "Async-MM runs with the coloured or sequential schedule");
    }
    return BD3MG_OK;
}

// The two H dp buffers, when H dp is kept (separable PSF, not Async-MM).
// Not having the memory is not an error: the direction pass then blurs both
// directions every sweep.
bd3mg_status ensure_hdp(bd3mg_problem p)
{
    if (p->hdp_every <= 0 || p->dense || p->prm.method == M_MM) return BD3MG_OK;
    const size_t need = 2 * p->hdp_slots * p->nx * p->ny * p->esz;
    if (need <= p->hdp_alloc) return BD3MG_OK;
    if (p->d_hdp) HIP_TRY(hipFree(p->d_hdp));
    p->d_hdp = nullptr;
    p->hdp_alloc = 0;
    p->hdp_valid = false;
    if (hipMalloc(&p->d_hdp, need) != hipSuccess) {
        p->d_hdp = nullptr;
        (void)hipGetLastError();
        return BD3MG_OK;
    }
    p->hdp_alloc = need;
    return BD3MG_OK;
}

// Direction-pass mode of sweep sw (counted from x^0): 0 blurs d1 and d2 and
// keeps no H dp; 1 blurs both and the update pass stores every block's H d'
// as the H dp of its next visit; 2 blurs d1 only and reads H dp.  Both
// directions are blurred again on every hdp_every-th sweep, so that the
// rounding the recurrence H dp' = u1 H d1 + u2 H dp carries does not build
// up; the choice depends on the sweep count only, so runs split into several
// calls, or checked at other sweeps, take the same modes.
int hdp_mode(bd3mg_problem p, bool noalloc, long long sw, bool valid)
{
    if (noalloc || p->dense || p->prm.method == M_MM || p->hdp_every <= 0 || !p->d_hdp) return 0;
    return (valid && sw % p->hdp_every != 0) ? 2 : 1;
}

// H d2 of a colour group's items in the H dp buffer of this sweep (the parity
// of cur) and the update's H d' into the other one, for modes 1 and 2.
template <typename T>
void hdp_state(bd3mg_problem p, DevState<T> &s, const bd3mg_problem_s::Group &gr, int mode)
{
    if (!mode) return;
    const size_t S = (size_t)p->nx * p->ny, span = p->hdp_slots * S;
    T *hb = (T *)p->d_hdp;
    s.hd[1] = hb + p->cur * span + (size_t)gr.dbase * S;
    s.hdw = hb + (p->cur ^ 1) * span + (size_t)gr.dbase * S;
}

bd3mg_status ensure_ready(bd3mg_problem p)
{
    if (!p->psf_set) return fail(BD3MG_ERR_STATE, "the PSF is not set");
    if (!p->data_set) return fail(BD3MG_ERR_STATE, "the data y is not set");
    ST_TRY(method_ready(p));
    ST_TRY(build_schedule(p));
    ST_TRY(ensure_hdp(p));
    if (!p->x_set) {
        HIP_TRY(hipMemcpyAsync(p->x, p->y, p->N * p->esz, hipMemcpyDeviceToDevice, p->stream));
        ST_TRY(zero_steps(p));
        p->x_set = true;
        p->q_stale = true;
        p->sweeps_done = 0;
    }
    if (!p->gnorm_ref_valid) {
        ST_TRY(ensure_tmp(p, 2));
        ST_TRY(refresh(p, p->y, p->tmp[1]));
        ST_TRY(eval_at(p, p->y, p->tmp[1], nullptr, &p->gnorm_ref));
        p->gnorm_ref_valid = true;
    }
    if (p->q_stale) {
        ST_TRY(refresh(p, p->x, p->q));
        p->q_stale = false;
    }
    return BD3MG_OK;
}

// Enqueue the passes of one launch group: gradient, direction, solve, update
// (hdp: the direction-pass mode of hdp_mode; colour groups only).
template <typename T>
bd3mg_status phase_t(bd3mg_problem p, const bd3mg_problem_s::Group &gr, bool prof, const int *stop, int hdp)
{
    DevState<T> s = dev_state<T>(p);
    s.stop = stop;
    // H d2 of the group's items (H dp, or blurred and stored by the direction
    // pass) in the buffer of this sweep, the pairs' H d' into the other one
    hdp_state<T>(p, s, gr, hdp);
    const Item *it = p->d_items;
    if (p->dense) {
        // general kernels: H^T r and grad f on S, H d1 and H d2 on S +- r_z by
        // the dense kernels, r += u1 H d1 + u2 H d2 elementwise
        if (prof) ST_TRY(prof_begin(p, BD3MG_K_GRAD, gr.bytes[0], false));
        HIP_TRY(dense_grad<T>(p, s, s.q, s.x, nullptr, it + gr.g_off, gr.g_cnt, GM_BLOCK, p->d_pg, true));
        if (prof) ST_TRY(prof_end(p));
        if (prof) ST_TRY(prof_begin(p, BD3MG_K_DIRS, gr.bytes[1]));
        HIP_TRY(launch_dense<T>(p->geom, p->prm, s, (const T *)p->d_pk, nullptr, nullptr, nullptr, it + gr.d_off,
                                gr.d_cnt, DM_DIRS, p->d_pd, p->stream));
        if (prof) ST_TRY(prof_end(p));
        if (prof) ST_TRY(prof_begin(p, BD3MG_K_SOLVE, gr.bytes[2]));
        HIP_TRY(launch_solve(p->prm, p->d_br + gr.br_off, gr.br_cnt, p->ntiles,
                             tiles_of(p->geom, p->geom.ty_dirs), p->d_pg, p->d_pd, p->d_u, p->d_info, stop,
                             p->stream));
        if (prof) ST_TRY(prof_end(p));
        if (prof) ST_TRY(prof_begin(p, BD3MG_K_UPDATE, gr.bytes[3]));
        HIP_TRY(launch_dense_update<T>(p->geom, s, it + gr.u_off, gr.u_cnt, p->d_pairs, p->d_u, p->stream));
        if (prof) ST_TRY(prof_end(p));
        return BD3MG_OK;
    }
    if (prof) ST_TRY(prof_begin(p, BD3MG_K_GRAD, gr.bytes[0]));
    HIP_TRY(launch_grad<T>(p->geom, p->prm, s, s.q, s.x, nullptr, it + gr.g_off, gr.g_cnt, GM_BLOCK,
                           p->d_pg, p->stream));
    if (prof) ST_TRY(prof_end(p));
    const double *u = p->d_u;
    if (p->prm.method == M_MM) {
        // Async-MM: v = A_S(x)^{-1} (-g_S) by inner conjugate gradients on
        // every block of the group, then d' = v applied as -g with u = (1, 0)
        const CgBufs<T> cb{(T *)p->mmv[0], (T *)p->mmv[1], (T *)p->mmv[2], (T *)p->mmv[3], (T *)p->mmv[4],
                           p->d_pg, p->d_pma, p->d_prr, p->d_cgs, p->d_info};
        const Item *gi = it + gr.g_off;
        if (prof) ST_TRY(prof_begin(p, BD3MG_K_SOLVE, 0.0, false));
        HIP_TRY(launch_cg<T>(CG_INIT, p->geom, s, gi, gr.g_cnt, cb, 0, p->tol_inner, p->stream));
        DevState<T> sp = s;  // H p from the direction pass (d1 = -p, d2 = p)
        sp.g = cb.p;
        sp.dp[0] = cb.p;
        DevState<T> sq = s;  // XY^T (H p) into qt
        sq.q = cb.qt;
        for (int i = 0; i < p->n_inner; ++i) {
            HIP_TRY(launch_dirs<T>(p->geom, p->prm, sp, p->d_units + gr.du_off, gr.du_cnt, p->d_pd, p->stream));
            HIP_TRY(launch_update<T>(p->geom, sq, it + gr.u_off, gr.u_cnt, p->d_pairs, p->d_u01, false,
                                     p->stream, 1));
            HIP_TRY(launch_majapply<T>(p->geom, p->prm, s, cb.qt, s.x, cb.p, cb.ap, gi, gr.g_cnt, p->d_pma,
                                       p->stream));
            HIP_TRY(launch_cg<T>(CG_VEC, p->geom, s, gi, gr.g_cnt, cb, i & 1, p->tol_inner, p->stream));
            HIP_TRY(launch_cg<T>(CG_DIR, p->geom, s, gi, gr.g_cnt, cb, i & 1, p->tol_inner, p->stream));
        }
        HIP_TRY(launch_cg<T>(CG_FINAL, p->geom, s, gi, gr.g_cnt, cb, 0, p->tol_inner, p->stream));
        if (prof) ST_TRY(prof_end(p));
        if (prof) ST_TRY(prof_begin(p, BD3MG_K_DIRS, gr.bytes[1]));
        HIP_TRY(launch_dirs<T>(p->geom, p->prm, s, p->d_units + gr.du_off, gr.du_cnt, p->d_pd, p->stream));
        if (prof) ST_TRY(prof_end(p));
        u = p->d_u10;
    } else {
        if (prof) ST_TRY(prof_begin(p, BD3MG_K_DIRS, hdp == 2 ? gr.bytes_one : gr.bytes[1]));
        HIP_TRY(launch_dirs<T>(p->geom, p->prm, s, p->d_units + gr.du_off, gr.du_cnt, p->d_pd, p->stream,
                               hdp == 2));
        if (prof) ST_TRY(prof_end(p));
        if (prof) ST_TRY(prof_begin(p, BD3MG_K_SOLVE, gr.bytes[2]));
        HIP_TRY(launch_solve(p->prm, p->d_br + gr.br_off, gr.br_cnt, p->ntiles,
                             tiles_of(p->geom, p->geom.ty_dirs), p->d_pg, p->d_pd, p->d_u, p->d_info, stop,
                             p->stream));
        if (prof) ST_TRY(prof_end(p));
    }
    if (prof) ST_TRY(prof_begin(p, BD3MG_K_UPDATE, gr.bytes[3] + (hdp ? gr.bytes_hdw : 0.0)));
    HIP_TRY(launch_update<T>(p->geom, s, it + gr.u_off, gr.u_cnt, p->d_pairs, u, gr.round, p->stream));
    if (prof) ST_TRY(prof_end(p));
    return BD3MG_OK;
}

bd3mg_status phase(bd3mg_problem p, const bd3mg_problem_s::Group &gr, bool prof,
                   const int *stop = nullptr, int hdp = 0)
{
    return p->prec == BD3MG_FP64 ? phase_t<double>(p, gr, prof, stop, hdp)
                                 : phase_t<float>(p, gr, prof, stop, hdp);
}

// One operator of the criterion on ti into to (tr, tr2: scratch volumes;
// tr2 only for grad f with general kernels, the problem's own scratch when
// null), with the solver's kernels: H directly; H^T as the adjoint in-slice
// blur of every slice followed by the z-stencil; grad f from
// q = XY^T (H ti - y).
template <typename T>
bd3mg_status apply_t(bd3mg_problem p, int op, T *ti, T *to, T *tr, T *tr2 = nullptr)
{
    DevState<T> s = dev_state<T>(p);
    if (p->dense) {
        const T *pk = (const T *)p->d_pk;
        if (op == BD3MG_OP_H) {
            HIP_TRY(launch_dense<T>(p->geom, p->prm, s, pk, ti, nullptr, to, p->d_vol, p->nz, DM_H, nullptr,
                                    p->stream));
        } else if (op == BD3MG_OP_HT) {
            HIP_TRY(launch_dense<T>(p->geom, p->prm, s, pk, ti, nullptr, to, p->d_vol, p->nz, DM_HT, nullptr,
                                    p->stream));
        } else {
            if (!tr2) ST_TRY(ensure_tmp(p, 4));
            HIP_TRY(launch_dense<T>(p->geom, p->prm, s, pk, ti, s.y, tr, p->d_vol, p->nz, DM_H, nullptr,
                                    p->stream));
            HIP_TRY(dense_grad<T>(p, s, tr, ti, to, p->d_vol, p->nz, GM_GRAD, nullptr, false, tr2));
        }
        return BD3MG_OK;
    }
    if (op == BD3MG_OP_H) {
        HIP_TRY(launch_H<T>(p->geom, s, ti, nullptr, to, p->d_vol, p->nz, nullptr, p->stream));
    } else if (op == BD3MG_OP_HT) {
        HIP_TRY(launch_blurT<T>(p->geom, s, ti, tr, p->d_vol, p->nz, p->stream));
        HIP_TRY(launch_grad<T>(p->geom, p->prm, s, tr, ti, to, p->d_vol, p->nz, GM_ZCOMB, nullptr,
                               p->stream));
    } else {
        HIP_TRY(launch_refresh<T>(p->geom, s, ti, tr, p->d_vol, p->nz, p->stream));
        HIP_TRY(launch_grad<T>(p->geom, p->prm, s, tr, ti, to, p->d_vol, p->nz, GM_GRAD, nullptr,
                               p->stream));
    }
    return BD3MG_OK;
}

bd3mg_status validate_handle(bd3mg_problem p)
{
    if (!p) return fail(BD3MG_ERR_ARG, "null problem handle");
    return BD3MG_OK;
}

// Scratch buffers of the run loop: partial sums, per-block coefficients, the
// stop-test control block and the stored directions.  bd3mg_run_noalloc
// points them into the per-device scratch array for one call and restores
// the problem's own afterwards.
struct WorkBuffers {
    double *pg, *pd, *pe, *pr, *u, *info, *sum;
    bd3mg_problem_s::Ctl *ctl;
    void *hd;
};

WorkBuffers work_of(bd3mg_problem p)
{
    return WorkBuffers{p->d_pg, p->d_pd, p->d_pe, p->d_pr, p->d_u, p->d_info, p->d_sum, p->d_ctl, p->d_hd};
}

void set_work(bd3mg_problem p, const WorkBuffers &w)
{
    p->d_pg = w.pg;
    p->d_pd = w.pd;
    p->d_pe = w.pe;
    p->d_pr = w.pr;
    p->d_u = w.u;
    p->d_info = w.info;
    p->d_sum = w.sum;
    p->d_ctl = w.ctl;
    p->d_hd = w.hd;
}

// Lay the run loop's scratch buffers of p out from base, each 256-byte
// aligned, with the sizes of the problem's own (schedule built); returns the
// bytes needed, and sets *w only when they fit in avail.
size_t carve_work(bd3mg_problem p, char *base, size_t avail, WorkBuffers *w)
{
    const size_t nb = p->nsl.size();
    const size_t nslot = (size_t)p->ntiles * p->nz;
    const size_t sizes[9] = {
        sizeof(bd3mg_problem_s::Ctl),
        2 * nb * sizeof(double),
        8 * nb * sizeof(double),
        (NQE + 1) * sizeof(double),
        (size_t)p->maxg * p->ntiles * NQG * sizeof(double),
        (size_t)p->maxd * tiles_of(p->geom, 16) * NQD * sizeof(double),
        nslot * NQE * sizeof(double),
        nslot * sizeof(double),
        2 * (size_t)p->hd_slots * p->nx * p->ny * p->esz,
    };
    size_t off[9], total = 0;
    for (int i = 0; i < 9; ++i) {
        off[i] = total;
        total += (sizes[i] + 255) / 256 * 256;
    }
    if (total <= avail && w) {
        w->ctl = (bd3mg_problem_s::Ctl *)(base + off[0]);
        w->u = (double *)(base + off[1]);
        w->info = (double *)(base + off[2]);
        w->sum = (double *)(base + off[3]);
        w->pg = (double *)(base + off[4]);
        w->pd = (double *)(base + off[5]);
        w->pe = (double *)(base + off[6]);
        w->pr = (double *)(base + off[7]);
        w->hd = base + off[8];
    }
    return total;
}

// The set-up of bd3mg_run without allocating: the schedule must be built
// already; x^0 = y, the reference gradient norm and q are formed in place.
bd3mg_status ensure_ready_noalloc(bd3mg_problem p)
{
    if (!p->psf_set) return fail(BD3MG_ERR_STATE, "the PSF is not set");
    if (!p->data_set) return fail(BD3MG_ERR_STATE, "the data y is not set");
    if (p->dense) return fail(BD3MG_ERR_STATE, "bd3mg_run_noalloc takes the separable PSF only");
    if (p->prm.method == M_MM) return fail(BD3MG_ERR_STATE, "bd3mg_run_noalloc does not run Async-MM");
    ST_TRY(method_ready(p));
    if (!p->blocks_set) return fail(BD3MG_ERR_STATE, "blocks are not set");
    if (p->sched_dirty)
        return fail(BD3MG_ERR_STATE, "the schedule is not built (bd3mg_get_schedule builds it)");
    if (!p->x_set) {
        HIP_TRY(hipMemcpyAsync(p->x, p->y, p->N * p->esz, hipMemcpyDeviceToDevice, p->stream));
        ST_TRY(zero_steps(p));
        p->x_set = true;
        p->q_stale = true;
        p->sweeps_done = 0;
    }
    if (!p->gnorm_ref_valid) {
        ST_TRY(refresh(p, p->y, p->q));
        ST_TRY(eval_at(p, p->y, p->q, nullptr, &p->gnorm_ref));
        p->gnorm_ref_valid = true;
        p->q_stale = true;
    }
    if (p->q_stale) {
        ST_TRY(refresh(p, p->x, p->q));
        p->q_stale = false;
    }
    return BD3MG_OK;
}

// Guard of the asynchronous rounds: the accepted state (x, every block's
// previous step, q) is copied to gsave, and back on a restore.
bd3mg_status guard_copy(bd3mg_problem p, bool save)
{
    for (int i = 0; i < 3; ++i)
        if (!p->gsave[i] && hipMalloc(&p->gsave[i], p->N * p->esz) != hipSuccess)
            return fail(BD3MG_ERR_NOMEM, "guard state volume of %zu bytes", p->N * p->esz);
    void *live[3] = {p->x, p->dpb[p->cur], p->q};
    for (int i = 0; i < 3; ++i)
        HIP_TRY(hipMemcpyAsync(save ? p->gsave[i] : live[i], save ? live[i] : p->gsave[i], p->N * p->esz,
                               hipMemcpyDeviceToDevice, p->stream));
    return BD3MG_OK;
}

// Inflation after the guard saw f increase: doubled, at least L / 16, at
// most the value mu = L (2 sqrt(tau) + 1), tau = nblocks - 1, under which
// Assumption C holds whatever the point.
bd3mg_status guard_raise(bd3mg_problem p)
{
    double L = 0.0;
    ST_TRY(bd3mg_lipschitz_bound(p, &L));
    const double cap = L * (2.0 * std::sqrt((double)p->nsl.size() - 1.0) + 1.0);
    p->prm.mu = std::min(cap, std::max(2.0 * p->prm.mu, L / 16.0));
    return BD3MG_OK;
}

double guard_cap(bd3mg_problem p)
{
    double L = 0.0;
    if (bd3mg_lipschitz_bound(p, &L) != BD3MG_OK) return 0.0;
    return L * (2.0 * std::sqrt((double)p->nsl.size() - 1.0) + 1.0);
}

// The run loop of bd3mg_run and bd3mg_run_noalloc.  noalloc: the set-up is
// done in place (no scratch volume is taken), a stop is confirmed on q
// rebuilt in place from x, and f at the end is formed in g (not read again
// before the next gradient pass writes it).
bd3mg_status run_impl(bd3mg_problem p, int max_sweeps, double grad_rtol, int check_every,
                      bd3mg_result *res, bool noalloc)
{
    ST_TRY(validate_handle(p));
    if (max_sweeps < 0) return fail(BD3MG_ERR_ARG, "max_sweeps < 0");
    if (check_every < BD3MG_CHECK_ADAPTIVE) return fail(BD3MG_ERR_ARG, "check_every < -1");
    const bool adaptive = check_every == BD3MG_CHECK_ADAPTIVE;
    if (adaptive && !(grad_rtol > 0.0)) return fail(BD3MG_ERR_ARG, "adaptive checks need grad_rtol > 0");
    const bool checking = grad_rtol > 0.0 || check_every > 0;
    if (grad_rtol > 0.0 && check_every == 0) check_every = max_sweeps > 0 ? max_sweeps : 1;
    ST_TRY(noalloc ? ensure_ready_noalloc(p) : ensure_ready(p));
    const double vol = (double)p->N * p->esz;
    // The stop test runs on the device: a check that meets the tolerance
    // raises a flag and every later pass returns without writing, so the host only
    // waits once per chunk of sweeps.
    constexpr int CHUNK = 16;
    const bool stopping = grad_rtol > 0.0;
    int *stop = stopping ? &p->d_ctl->stop : nullptr;
    const double thr = stopping ? grad_rtol * p->gnorm_ref : -1.0;
    HIP_TRY(hipMemsetAsync(p->d_ctl, 0, sizeof(bd3mg_problem_s::Ctl), p->stream));
    HIP_TRY(hipEventRecord(p->ev0, p->stream));
    const int cur0 = p->cur;
    const long long sweeps0 = p->sweeps_done;
    int done = max_sweeps;
    bool conv = false;
    // Guard of the asynchronous rounds (BD3MG_OPT_ROUND_GUARD): every
    // round_guard sweeps f is evaluated; when it rose above the last accepted
    // value the state goes back to the accepted one and the inflation is
    // raised.  lost counts the sweeps run and then discarded, so the state's
    // own sweep count is s - lost.
    const bool guard = !noalloc && p->schedule == BD3MG_SCHED_ROUND && p->round_guard > 0;
    const double slack = p->prec == BD3MG_FP32 ? 4e-9 : 1e-13;
    int lost = 0, s_acc = 0, g_cur = p->cur;
    double f_acc = 0.0;
    p->guard_trips = 0;
    if (guard) {
        ST_TRY(eval_at(p, p->x, p->q, &f_acc, nullptr));
        ST_TRY(guard_copy(p, true));
    }
    bd3mg_problem_s::Ctl ctl{0, 0, NAN};
    // adaptive checks: the last two checks (sweep, ||grad f||)
    int sa = -1, sb = -1;
    double ga = 0.0, gb = 0.0;
    for (int s = 0; s < max_sweeps;) {
        int end = std::min(max_sweeps, s + CHUNK);
        bool every = true;  // adaptive: check after every sweep of the chunk, else after its last
        if (adaptive) {
            if (sb < 0) {
                end = s + 1;  // a first check after one sweep
            } else if (sa >= 0 && ga > 0.0 && gb > 0.0 && gb < ga && gb > thr) {
                // ||grad f|| decreasing: where log ||grad f|| reaches log thr
                // on the line through the last two checks
                const double rate = std::log(gb / ga) / (double)(sb - sa);
                const double ahead = std::log(thr / gb) / rate;
                if (ahead > 8.0) {
                    // far from it: half the predicted distance, one check at the end
                    const int len = (int)std::min(256.0, 0.5 * ahead);
                    end = std::min(max_sweeps, s + len);
                    every = false;
                }
            } else if (gb > thr) {
                every = false;  // no trend yet: one check at the end of the chunk
            }
        }
        for (; s < end; ++s) {
            const int hm = hdp_mode(p, noalloc, sweeps0 + s, p->hdp_valid);
            for (int c = 0; c < p->ncolors; ++c) ST_TRY(phase(p, p->groups[c], p->profile, stop, hm));
            p->hdp_valid = hm != 0;
            p->cur ^= 1;
            const long long sw = sweeps0 + s + 1;
            if (p->refresh_every > 0 && (sw % p->refresh_every) == 0) {
                ST_TRY(prof_begin(p, BD3MG_K_EVAL, 3.0 * vol));
                ST_TRY(refresh(p, p->x, p->q, stop));
                ST_TRY(prof_end(p));
            }
            // (check_every is 0 when nothing is checked: no modulo then)
            const bool due = checking && (adaptive ? (every || s + 1 == end)
                                                   : (((s + 1) % check_every) == 0 || s + 1 == max_sweeps));
            if (due) {
                ST_TRY(prof_begin(p, BD3MG_K_EVAL, 2.0 * vol, false));
                ST_TRY(check(p, thr, s + 1, stop));
                ST_TRY(prof_end(p));
            }
        }
        if (checking) {
            HIP_TRY(hipMemcpyAsync(&ctl, p->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost, p->stream));
            HIP_TRY(hipStreamSynchronize(p->stream));
            if (ctl.stop) {
                // The device test read the maintained residual q, which drifts
                // from XY^T (H x - y) by rounding between refreshes.  Confirm
                // on a residual rebuilt from x (a scratch volume, so the
                // state and the bitwise equality of chained runs are kept);
                // if the rebuilt gradient is still above the threshold, take
                // the rebuilt residual as q and continue from the stop sweep.
                const int ss = ctl.stop_sweep;
                p->cur = cur0 ^ ((ss - lost) & 1);
                double gfresh = 0.0;
                void *qf = p->q;  // rebuilt in place when nothing may be allocated
                if (!noalloc) {
                    ST_TRY(ensure_tmp(p, 2));
                    qf = p->tmp[1];
                }
                ST_TRY(refresh(p, p->x, qf));
                ST_TRY(eval_at(p, p->x, qf, nullptr, &gfresh));
                if (gfresh <= thr) {
                    done = ss;
                    conv = true;
                    break;
                }
                if (qf != p->q)
                    HIP_TRY(hipMemcpyAsync(p->q, qf, vol, hipMemcpyDeviceToDevice, p->stream));
                HIP_TRY(hipMemsetAsync(p->d_ctl, 0, sizeof(bd3mg_problem_s::Ctl), p->stream));
                ctl = bd3mg_problem_s::Ctl{0, 0, gfresh};
                s = ss;
                if (ss >= max_sweeps) break;
            }
            if (adaptive) {
                sa = sb;
                ga = gb;
                sb = s;
                gb = ctl.gnorm;
            }
        }
        if (guard && s - s_acc >= p->round_guard) {
            double fs = 0.0;
            ST_TRY(eval_at(p, p->x, p->q, &fs, nullptr));
            if (fs <= f_acc + slack * std::fabs(f_acc) || p->prm.mu >= guard_cap(p)) {
                ST_TRY(guard_copy(p, true));
                f_acc = fs;
                s_acc = s;
                g_cur = p->cur;
            } else {
                // back to the accepted state, with more curvature
                p->cur = g_cur;
                ST_TRY(guard_copy(p, false));
                lost += s - s_acc;
                s_acc = s;
                p->hdp_valid = false;
                ST_TRY(guard_raise(p));
                ++p->guard_trips;
                sa = sb = -1;
                HIP_TRY(hipMemsetAsync(p->d_ctl, 0, sizeof(bd3mg_problem_s::Ctl), p->stream));
                ctl = bd3mg_problem_s::Ctl{0, 0, NAN};
            }
        }
        if (p->pending.size() > 4096) ST_TRY(prof_collect(p));
    }
    p->cur = cur0 ^ ((done - lost) & 1);
    p->sweeps_done = sweeps0 + done - lost;
    HIP_TRY(hipEventRecord(p->ev1, p->stream));
    double gn = ctl.gnorm, f = NAN;
    if (checking) {
        // f and ||grad f|| of the returned x from a residual rebuilt from x
        if (noalloc) {
            ST_TRY(refresh(p, p->x, p->q));
            ST_TRY(eval_at(p, p->x, p->q, &f, &gn, p->g));
        } else {
            ST_TRY(ensure_tmp(p, 2));
            ST_TRY(refresh(p, p->x, p->tmp[1]));
            ST_TRY(eval_at(p, p->x, p->tmp[1], &f, &gn));
        }
    }
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

}  // namespace

bd3mg_status bd3mg::problem_view(bd3mg_problem p, ProblemView *v)
{
    ST_TRY(validate_handle(p));
    *v = ProblemView{p->nx, p->ny, p->nz, p->prec, p->data_set, p->y, p->stream};
    return BD3MG_OK;
}

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

bd3mg_status bd3mg_create(int nx, int ny, int nz, int precision, void *hip_stream, bd3mg_problem *out)
{
    if (!out) return fail(BD3MG_ERR_ARG, "null output handle");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(BD3MG_ERR_ARG, "dimensions must be >= 1");
    if (precision != BD3MG_FP64 && precision != BD3MG_FP32)
        return fail(BD3MG_ERR_ARG, "unknown precision %d", precision);
    // in-slice byte offsets are formed in 32 bits by the kernels
    if ((size_t)nx * ny * (precision == BD3MG_FP64 ? 8 : 4) >= ((size_t)1 << 31))
        return fail(BD3MG_ERR_ARG, "a slice of %d x %d exceeds 2 GiB", nx, ny);
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
    {
        const int ty = precision == BD3MG_FP64 ? 16 : 32;
        p->geom.ty_dirs = p->geom.ty_update = p->geom.ty_aux = ty;
    }
    auto bail = [&](bd3mg_status st, const char *what) {
        bd3mg_destroy(p);
        return fail(st, "%s", what);
    };
    if (hipGetDevice(&p->device) != hipSuccess) return bail(BD3MG_ERR_HIP, "no current HIP device");
    if (hip_stream) {
        p->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(BD3MG_ERR_HIP, "stream creation failed");
        p->own_stream = true;
    }
    if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
        return bail(BD3MG_ERR_HIP, "event creation failed");
    p->ntiles = p->geom.ntx * p->geom.nty;
    void **vols[] = {&p->x, &p->y, &p->q, &p->g, &p->dpb[0], &p->dpb[1]};
    for (void **v : vols)
        if (hipMalloc(v, p->N * p->esz) != hipSuccess) return bail(BD3MG_ERR_NOMEM, "volume allocation failed");
    // every slice of the volume as a work item, and the evaluation sums
    std::vector<Item> vol;
    for (int k = 0; k < nz; ++k) vol.push_back(Item{k, -1, 0, nz, 0, 0});
    const size_t nslot = (size_t)p->ntiles * nz;
    if (hipMalloc(&p->d_vol, vol.size() * sizeof(Item)) != hipSuccess ||
        hipMalloc(&p->d_pe, nslot * NQE * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->d_pr, nslot * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->d_sum, (NQE + 1) * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->d_ctl, sizeof(bd3mg_problem_s::Ctl)) != hipSuccess)
        return bail(BD3MG_ERR_NOMEM, "tables");
    if (hipMemcpy(p->d_vol, vol.data(), vol.size() * sizeof(Item), hipMemcpyHostToDevice) != hipSuccess)
        return bail(BD3MG_ERR_HIP, "item upload failed");
    if (zero_steps(p) != BD3MG_OK) return bail(BD3MG_ERR_HIP, "clearing steps failed");
    *out = p;
    return BD3MG_OK;
}

bd3mg_status bd3mg_destroy(bd3mg_problem p)
{
    if (!p) return BD3MG_OK;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    void *bufs[] = {p->x, p->y, p->q, p->g, p->dpb[0], p->dpb[1], p->tmp[0], p->tmp[1], p->tmp[2], p->tmp[3],
                    p->d_pk, p->d_ones, p->d_hts,
                    p->d_gx, p->d_gy, p->d_gz, p->d_items, p->d_br, p->d_vol, p->d_sblk, p->d_pg, p->d_pd,
                    p->d_pe, p->d_pr, p->d_u, p->d_info, p->d_sum, p->d_ctl, p->d_pairs, p->d_hd,
                    p->d_units, p->d_hdp, p->gsave[0], p->gsave[1], p->gsave[2]};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    void *mm[] = {p->mmv[0], p->mmv[1], p->mmv[2], p->mmv[3], p->mmv[4], p->d_pma, p->d_prr, p->d_cgs,
                  p->d_u01, p->d_u10};
    for (void *b : mm)
        if (b) (void)hipFree(b);
    for (auto &q : p->pending) {
        (void)hipEventDestroy(q.a);
        (void)hipEventDestroy(q.b);
    }
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->stream && p->own_stream) (void)hipStreamDestroy(p->stream);
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
    // in-slice tables are stored centred in 2R + 1 taps, R = max(rx, ry, 1)
    const int R = std::max(1, std::max(kx / 2, ky / 2)), KR = 2 * R + 1;
    std::vector<double> px((size_t)p->nz * KR, 0.0), py((size_t)p->nz * KR, 0.0);
    for (int z = 0; z < p->nz; ++z) {
        for (int a = 0; a < kx; ++a) px[(size_t)z * KR + R - kx / 2 + a] = gx[(size_t)z * kx + a];
        for (int a = 0; a < ky; ++a) py[(size_t)z * KR + R - ky / 2 + a] = gy[(size_t)z * ky + a];
    }
    const double *src[3] = {px.data(), py.data(), gz};
    const int ks[3] = {KR, KR, kz};
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
    p->hgx.assign(gx, gx + (size_t)p->nz * kx);
    p->hgy.assign(gy, gy + (size_t)p->nz * ky);
    p->hgz.assign(gz, gz + (size_t)p->nz * kz);
    p->geom.R = R;
    p->kx = kx;
    p->ky = ky;
    p->kz = kz;
    p->geom.rx = kx / 2;
    p->geom.ry = ky / 2;
    p->geom.rz = kz / 2;
    p->dense = false;
    p->psf_set = true;
    p->q_stale = true;
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
    p->prm = Params{lambda, delta, eta, kappa, xmin, xmax, p->prm.mu, p->prm.method, p->prm.lip, p->prm.tv3d};
    p->gnorm_ref_valid = false;
    if (kappa_changed) p->sched_dirty = true;
    return BD3MG_OK;
}

bd3mg_status bd3mg_round_guard_info(bd3mg_problem p, int *trips, double *mu)
{
    ST_TRY(validate_handle(p));
    if (trips) *trips = p->guard_trips;
    if (mu) *mu = p->prm.mu;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_inflation(bd3mg_problem p, double mu)
{
    ST_TRY(validate_handle(p));
    if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(BD3MG_ERR_ARG, "mu must be finite and >= 0");
    p->prm.mu = mu;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_tv3d(bd3mg_problem p, int on)
{
    ST_TRY(validate_handle(p));
    if (on != 0 && on != 1) return fail(BD3MG_ERR_ARG, "on must be 0 or 1, got %d", on);
    if (on && p->prm.method == M_MM)
        return fail(BD3MG_ERR_STATE, "Async-MM runs with the total variation of the slices");
    if (on != p->prm.tv3d) {
        p->prm.tv3d = on;
        p->gnorm_ref_valid = false;
        p->sched_dirty = true;  // the colouring gap and the direction items depend on it
    }
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_method(bd3mg_problem p, int method, double lip, int n_inner, double tol_inner)
{
    ST_TRY(validate_handle(p));
    if (method < BD3MG_METHOD_BD3MG || method > BD3MG_METHOD_ASYNC_MM)
        return fail(BD3MG_ERR_ARG, "unknown method %d", method);
    if (!std::isfinite(lip)) return fail(BD3MG_ERR_ARG, "L must be finite");
    if (method == BD3MG_METHOD_ASYNC_MM && (n_inner < 1 || n_inner > 10000))
        return fail(BD3MG_ERR_ARG, "Async-MM needs 1 <= n_inner <= 10000, got %d", n_inner);
    if (!(tol_inner >= 0.0) || !std::isfinite(tol_inner)) return fail(BD3MG_ERR_ARG, "tol_inner must be >= 0");
    if (method == BD3MG_METHOD_ASYNC_MM && p->dense)
        return fail(BD3MG_ERR_STATE, "Async-MM runs with the separable PSF");
    if (method == BD3MG_METHOD_ASYNC_MM && p->prm.tv3d)
        return fail(BD3MG_ERR_STATE, "Async-MM runs with the total variation of the slices");
    const bool to_mm = method == BD3MG_METHOD_ASYNC_MM && p->prm.method != M_MM;
    p->prm.method = method;
    p->lip_given = lip;
    p->n_inner = n_inner;
    p->tol_inner = tol_inner;
    if (to_mm) p->sched_dirty = true;  // the inner solve's buffers are sized with the schedule
    return BD3MG_OK;
}

bd3mg_status bd3mg_psf_rotated_gaussian(int nz, int kxy, int kz, const double *sx, const double *sy,
                                        const double *theta, const double *sz, double *out)
{
    if (nz < 1 || kxy < 1 || kz < 1 || (kxy % 2) == 0 || (kz % 2) == 0)
        return fail(BD3MG_ERR_ARG, "need nz >= 1 and odd kernel sizes");
    if (!sx || !sy || !theta || !sz || !out) return fail(BD3MG_ERR_ARG, "null pointer");
    for (int z = 0; z < nz; ++z)
        if (!(sx[z] > 0.0) || !(sy[z] > 0.0) || !(sz[z] > 0.0) || !std::isfinite(sx[z]) ||
            !std::isfinite(sy[z]) || !std::isfinite(sz[z]) || !std::isfinite(theta[z]))
            return fail(BD3MG_ERR_ARG, "widths must be positive and finite, the angle finite (slice %d)", z);
    const int r = kxy / 2, rz = kz / 2;
    const size_t per = (size_t)kz * kxy * kxy;
    for (int z = 0; z < nz; ++z) {
        double *o = out + (size_t)z * per;
        const double c = std::cos(theta[z]), sn = std::sin(theta[z]);
        const double ax = 0.5 / (sx[z] * sx[z]), ay = 0.5 / (sy[z] * sy[z]), az = 0.5 / (sz[z] * sz[z]);
        double tot = 0.0;
        size_t q = 0;
        for (int t = -rz; t <= rz; ++t)
            for (int b = -r; b <= r; ++b)
                for (int a = -r; a <= r; ++a, ++q) {
                    // coordinates along and across the rotated axis
                    const double u = c * a + sn * b, v = c * b - sn * a;
                    o[q] = std::exp(-(ax * u * u + ay * v * v + az * t * t));
                    tot += o[q];
                }
        for (q = 0; q < per; ++q) o[q] /= tot;
    }
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_psf_dense(bd3mg_problem p, int kx, int ky, int kz, const double *P)
{
    ST_TRY(validate_handle(p));
    for (int k : {kx, ky})
        if (k < 1 || (k % 2) == 0 || k > 2 * RDMAX + 1)
            return fail(BD3MG_ERR_ARG, "in-slice kernel sizes must be odd, 1..%d (got %d)", 2 * RDMAX + 1, k);
    if (kz < 1 || (kz % 2) == 0 || kz > KZDMAX)
        return fail(BD3MG_ERR_ARG, "kz must be odd, 1..%d (got %d)", KZDMAX, kz);
    if (!P) return fail(BD3MG_ERR_ARG, "null kernel table");
    const size_t per = (size_t)kz * ky * kx;
    ST_TRY(check_finite(P, (size_t)p->nz * per, "P"));
    // stored centred in (2R + 1) x (2R + 1) per tap plane, R = max(rx, ry, 1)
    const int R = std::max(1, std::max(kx / 2, ky / 2)), KR = 2 * R + 1;
    const size_t n = (size_t)p->nz * kz * KR * KR;
    std::vector<double> t(n, 0.0);
    for (int z = 0; z < p->nz; ++z)
        for (int c = 0; c < kz; ++c)
            for (int b = 0; b < ky; ++b)
                for (int a = 0; a < kx; ++a)
                    t[(((size_t)z * kz + c) * KR + (R - ky / 2 + b)) * KR + (R - kx / 2 + a)] =
                        P[(((size_t)z * kz + c) * ky + b) * kx + a];
    if (p->d_pk) HIP_TRY(hipFree(p->d_pk));
    if (p->d_ones) HIP_TRY(hipFree(p->d_ones));
    p->d_pk = p->d_ones = nullptr;
    if (hipMalloc(&p->d_pk, n * p->esz) != hipSuccess || hipMalloc(&p->d_ones, (size_t)p->nz * p->esz) != hipSuccess)
        return fail(BD3MG_ERR_NOMEM, "kernel table");
    std::vector<double> ones((size_t)p->nz, 1.0);
    if (p->prec == BD3MG_FP64) {
        HIP_TRY(hipMemcpy(p->d_pk, t.data(), n * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_ones, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(t.begin(), t.end()), o(ones.begin(), ones.end());
        HIP_TRY(hipMemcpy(p->d_pk, f.data(), n * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_ones, o.data(), o.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    p->hpk.assign(P, P + (size_t)p->nz * per);
    p->geom.R = R;
    p->kx = kx;
    p->ky = ky;
    p->kz = kz;
    p->geom.rx = kx / 2;
    p->geom.ry = ky / 2;
    p->geom.rz = kz / 2;
    p->dense = true;
    p->psf_set = true;
    p->q_stale = true;
    p->gnorm_ref_valid = false;
    p->sched_dirty = true;
    return BD3MG_OK;
}

bd3mg_status bd3mg_lipschitz_bound(bd3mg_problem p, double *L)
{
    ST_TRY(validate_handle(p));
    if (!L) return fail(BD3MG_ERR_ARG, "null output");
    if (!p->psf_set) return fail(BD3MG_ERR_STATE, "the PSF is not set");
    // the tables in the storage precision, as the operator uses them
    auto st = [&](double v) { return std::fabs(p->prec == BD3MG_FP64 ? v : (double)(float)v); };
    const int rz = p->kz / 2, nz = p->nz;
    if (p->dense) {
        // row sums of |H| bounded by sum |P_k| of an output slice, column sums
        // by what an input slice s gathers, sum_c sum_{b,a} |P_{s+c}[c][b][a]|
        const size_t kk = (size_t)p->ky * p->kx;
        double rmax = 0.0, cmax = 0.0;
        for (int k = 0; k < nz; ++k) {
            double r = 0.0, c = 0.0;
            for (int t = -rz; t <= rz; ++t)
                for (size_t q = 0; q < kk; ++q) {
                    r += st(p->hpk[((size_t)k * p->kz + t + rz) * kk + q]);
                    if (k + t >= 0 && k + t < nz) c += st(p->hpk[((size_t)(k + t) * p->kz + t + rz) * kk + q]);
                }
            rmax = std::max(rmax, r);
            cmax = std::max(cmax, c);
        }
        const Params &q = p->prm;
        *L = rmax * cmax + 2.0 * q.eta + (q.tv3d ? 12.0 : 8.0) * q.lambda / q.delta + 8.0 * q.kappa;
        return BD3MG_OK;
    }
    double rmax = 0.0, cmax = 0.0, sx = 0.0, sy = 0.0;
    for (int k = 0; k < nz; ++k) {
        double r = 0.0, c = 0.0, ax = 0.0, ay = 0.0;
        for (int t = -rz; t <= rz; ++t) {
            if (k - t >= 0 && k - t < nz) r += st(p->hgz[(size_t)k * p->kz + t + rz]);
            if (k + t >= 0 && k + t < nz) c += st(p->hgz[(size_t)(k + t) * p->kz + t + rz]);
        }
        for (int a = 0; a < p->kx; ++a) ax += st(p->hgx[(size_t)k * p->kx + a]);
        for (int a = 0; a < p->ky; ++a) ay += st(p->hgy[(size_t)k * p->ky + a]);
        rmax = std::max(rmax, r);
        cmax = std::max(cmax, c);
        sx = std::max(sx, ax);
        sy = std::max(sy, ay);
    }
    const Params &q = p->prm;
    *L = rmax * cmax * sx * sx * sy * sy + 2.0 * q.eta + (q.tv3d ? 12.0 : 8.0) * q.lambda / q.delta +
         8.0 * q.kappa;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_data(bd3mg_problem p, const void *y, int on_device)
{
    ST_TRY(validate_handle(p));
    if (!y) return fail(BD3MG_ERR_ARG, "null data");
    ST_TRY(upload(p, p->y, y, on_device));
    p->data_set = true;
    p->q_stale = true;
    p->gnorm_ref_valid = false;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_blocks(bd3mg_problem p, int nblocks, const int *nslices, int schedule)
{
    ST_TRY(validate_handle(p));
    if (nblocks < 1 || !nslices) return fail(BD3MG_ERR_ARG, "need nblocks >= 1 and slice counts");
    if (schedule != BD3MG_SCHED_COLORED && schedule != BD3MG_SCHED_SEQUENTIAL &&
        schedule != BD3MG_SCHED_ROUND)
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
    p->q_stale = true;
    p->sweeps_done = 0;
    return BD3MG_OK;
}

bd3mg_status bd3mg_run(bd3mg_problem p, int max_sweeps, double grad_rtol, int check_every,
                       bd3mg_result *res)
{
    return run_impl(p, max_sweeps, grad_rtol, check_every, res, false);
}

bd3mg_status bd3mg_run_noalloc(bd3mg_problem p, int max_sweeps, double grad_rtol, int check_every,
                               bd3mg_result *res)
{
    ST_TRY(validate_handle(p));
    if (!p->blocks_set || p->sched_dirty || p->dense || !p->psf_set || !p->data_set || p->prm.method == M_MM)
        return ensure_ready_noalloc(p);  // fails, naming what is missing
    void *base = nullptr;
    HIP_TRY(scratch_base(p->device, &base));
    WorkBuffers w{};
    const size_t need = carve_work(p, (char *)base, SCRATCH_BYTES, &w);
    if (need > SCRATCH_BYTES)
        return fail(BD3MG_ERR_ARG, "this problem needs %zu bytes of scratch; bd3mg_run_noalloc has %zu",
                    need, SCRATCH_BYTES);
    const WorkBuffers own = work_of(p);
    const bool prof = p->profile;
    set_work(p, w);
    p->profile = false;  // event records would create events
    const bd3mg_status st = run_impl(p, max_sweeps, grad_rtol, check_every, res, true);
    p->profile = prof;
    set_work(p, own);
    return st;
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

bd3mg_status bd3mg_get_state(bd3mg_problem p, void *x, void *dprev, void *q, long long *sweeps,
                             int on_device)
{
    ST_TRY(validate_handle(p));
    if (!p->x_set) return fail(BD3MG_ERR_STATE, "no iterate yet");
    if (q && p->q_stale) ST_TRY(ensure_ready(p));
    if (x) ST_TRY(download(p, x, p->x, on_device));
    if (dprev) ST_TRY(download(p, dprev, p->dpb[p->cur], on_device));
    if (q) ST_TRY(download(p, q, p->q, on_device));
    if (sweeps) *sweeps = p->sweeps_done;
    return BD3MG_OK;
}

bd3mg_status bd3mg_set_state(bd3mg_problem p, const void *x, const void *dprev, const void *q,
                             long long sweeps, int on_device)
{
    ST_TRY(validate_handle(p));
    if (!x || !dprev) return fail(BD3MG_ERR_ARG, "null state");
    if (sweeps < 0) return fail(BD3MG_ERR_ARG, "sweeps < 0");
    ST_TRY(upload(p, p->x, x, on_device));
    ST_TRY(upload(p, p->dpb[p->cur], dprev, on_device));
    p->hdp_valid = false;
    p->x_set = true;
    if (q) {
        ST_TRY(upload(p, p->q, q, on_device));
        p->q_stale = false;
    } else {
        p->q_stale = true;
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
    case BD3MG_OPT_ROUND_GUARD:
        if (value < 0) return fail(BD3MG_ERR_ARG, "guard interval < 0");
        p->round_guard = value;
        return BD3MG_OK;
    case BD3MG_OPT_HDP_EVERY:
        if (value < 0) return fail(BD3MG_ERR_ARG, "H dp interval < 0");
        p->hdp_every = value;
        p->hdp_valid = false;
        return BD3MG_OK;
    case BD3MG_OPT_TILE_ROWS_DIRS:
    case BD3MG_OPT_TILE_ROWS_UPDATE:
    case BD3MG_OPT_TILE_ROWS_AUX: {
        if (value != 16 && !(value == 32 && p->prec == BD3MG_FP32))
            return fail(BD3MG_ERR_ARG, "tile rows must be 16 (or 32 in FP32), got %lld", value);
        int *t = option == BD3MG_OPT_TILE_ROWS_DIRS     ? &p->geom.ty_dirs
                 : option == BD3MG_OPT_TILE_ROWS_UPDATE ? &p->geom.ty_update
                                                        : &p->geom.ty_aux;
        *t = (int)value;
        return BD3MG_OK;
    }
    case BD3MG_OPT_STREAM_STORES:
        if (value < -1 || value > 1) return fail(BD3MG_ERR_ARG, "stream stores must be -1, 0 or 1");
        p->stream_stores = (int)value;
        return BD3MG_OK;
    case BD3MG_OPT_DIRS_SLICES:
        if (value < 0 || value > 2) return fail(BD3MG_ERR_ARG, "direction slices must be 0, 1 or 2");
        p->dirs_slices = (int)value;
        p->sched_dirty = true;
        return BD3MG_OK;
    default:
        return fail(BD3MG_ERR_ARG, "unknown option %d", option);
    }
}

bd3mg_status bd3mg_autotune(bd3mg_problem p, int sweeps, int *chosen, double *ms_out)
{
    ST_TRY(validate_handle(p));
    if (sweeps < 1) return fail(BD3MG_ERR_ARG, "sweeps < 1");
    ST_TRY(ensure_ready(p));
    ST_TRY(ensure_tmp(p, 3));
    // save the state
    const size_t vb = p->N * p->esz;
    HIP_TRY(hipMemcpyAsync(p->tmp[0], p->x, vb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->tmp[1], p->dpb[p->cur], vb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->tmp[2], p->q, vb, hipMemcpyDeviceToDevice, p->stream));
    const int cur0 = p->cur;
    const long long sw0 = p->sweeps_done;
    const bool prof0 = p->profile;
    p->profile = false;
    std::vector<int> cand = {16};
    if (p->prec == BD3MG_FP32) cand.push_back(32);
    std::vector<int> cand_u = cand;
    if (p->dense) cand_u = {p->geom.ty_update};  // the general-kernel passes use the direction tile only
    std::vector<std::pair<int, int>> combos;
    for (int td : cand)
        for (int tu : cand_u) combos.emplace_back(td, tu);
    // a warm-up at the current tiles first (clocks and caches settle), then
    // every candidate twice, in forward and then reverse order, keeping its
    // faster time: a single pass in a fixed order favours the later ones
    ST_TRY(bd3mg_run(p, sweeps, 0.0, 0, nullptr));
    std::vector<double> tmin(combos.size(), -1.0);
    for (int rep = 0; rep < 2; ++rep)
        for (size_t c0 = 0; c0 < combos.size(); ++c0) {
            const size_t c = rep ? combos.size() - 1 - c0 : c0;
            p->geom.ty_dirs = combos[c].first;
            p->geom.ty_update = combos[c].second;
            bd3mg_result r;
            ST_TRY(bd3mg_run(p, 1, 0.0, 0, nullptr));
            ST_TRY(bd3mg_run(p, sweeps, 0.0, 0, &r));
            const double t = r.seconds * 1e3 / sweeps;
            if (tmin[c] < 0.0 || t < tmin[c]) tmin[c] = t;
        }
    size_t bc = 0;
    for (size_t c = 1; c < combos.size(); ++c)
        if (tmin[c] < tmin[bc]) bc = c;
    const double best = tmin[bc];
    const int bd = combos[bc].first, bu = combos[bc].second;
    p->geom.ty_dirs = bd;
    p->geom.ty_update = bu;
    p->profile = prof0;
    // restore the state (H dp is blurred afresh on the next sweep)
    p->cur = cur0;
    p->hdp_valid = false;
    HIP_TRY(hipMemcpyAsync(p->x, p->tmp[0], vb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->dpb[p->cur], p->tmp[1], vb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->q, p->tmp[2], vb, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->sweeps_done = sw0;
    if (chosen) {
        chosen[0] = bd;
        chosen[1] = bu;
    }
    if (ms_out) *ms_out = best;
    return BD3MG_OK;
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
    ST_TRY(refresh(p, p->x, p->q));
    return eval_at(p, p->x, p->q, f, grad_norm);
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
        ST_TRY(apply_t<double>(p, op, (double *)p->tmp[0], (double *)p->tmp[1], (double *)p->tmp[2]));
    } else {
        ST_TRY(apply_t<float>(p, op, (float *)p->tmp[0], (float *)p->tmp[1], (float *)p->tmp[2]));
    }
    return download(p, out, p->tmp[1], on_device);
}

bd3mg_status bd3mg_block_step(bd3mg_problem p, int block, double *info)
{
    ST_TRY(validate_handle(p));
    ST_TRY(ensure_ready(p));
    const int nb = (int)p->nsl.size();
    if (block < 0 || block >= nb) return fail(BD3MG_ERR_ARG, "block %d out of range", block);
    ST_TRY(phase(p, p->groups[p->ncolors + block], false));
    p->hdp_valid = false;  // this block's step changed outside the sweep order
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
        // every launch shape; the first launch of each warms up
        for (int v = 0; v < COPY_VARIANTS && rc == BD3MG_OK; ++v)
            for (int it = 0; it <= iters && rc == BD3MG_OK; ++it) {
                float t = 0.f;
                if (hipEventRecord(e0, st) != hipSuccess || launch_copy(a, b, n16, v, st) != hipSuccess ||
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

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct bd3mg_batch_s {
    std::vector<bd3mg_problem> probs;
    hipStream_t s0 = nullptr;
    hipEvent_t fork = nullptr, ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> join;
    // Graphs of two sweeps, kept for the states they were captured in: per
    // problem -1 when inactive, else its previous-step buffer (cur) and the
    // direction-pass modes of the two sweeps (H dp kept or not).  A batch
    // whose problems advance together needs two: the pair that blurs both
    // directions again and the others.
    struct Graph {
        std::vector<int> key;
        bool fused = false;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        // fused launches: the per-problem argument sets and owner tables of
        // every (sweep of two, colour index, pass)
        void *d_fa = nullptr;
        unsigned char *d_owner = nullptr;
        unsigned long long used = 0;
    };
    std::vector<Graph> graphs;
    unsigned long long tick = 0;
    int mode = BD3MG_BATCH_AUTO;
};

namespace {

void graph_free(bd3mg_batch_s::Graph &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.d_fa) (void)hipFree(g.d_fa);
    if (g.d_owner) (void)hipFree(g.d_owner);
    g = bd3mg_batch_s::Graph{};
}

void batch_drop_graph(bd3mg_batch b)
{
    for (auto &g : b->graphs) graph_free(g);
    b->graphs.clear();
}

// Direction-pass modes of a problem's next two sweeps (see hdp_mode).
void pair_modes(bd3mg_problem p, int m[2])
{
    m[0] = hdp_mode(p, false, p->sweeps_done, p->hdp_valid);
    m[1] = hdp_mode(p, false, p->sweeps_done + 1, m[0] != 0);
}

std::vector<int> graph_key(bd3mg_batch b, const std::vector<char> &active)
{
    std::vector<int> key(b->probs.size(), -1);
    for (size_t i = 0; i < b->probs.size(); ++i) {
        if (!active[i]) continue;
        int m[2];
        pair_modes(b->probs[i], m);
        key[i] = b->probs[i]->cur | (m[0] << 1) | (m[1] << 3);
    }
    return key;
}

// Capture two sweeps of every active problem, each problem on its own stream
// between a fork and a join event of the batch stream, into one graph.
bd3mg_status batch_capture(bd3mg_batch b, const std::vector<char> &active, bd3mg_batch_s::Graph &out)
{
    HIP_TRY(hipStreamBeginCapture(b->s0, hipStreamCaptureModeRelaxed));
    bd3mg_status st = BD3MG_OK;
    if (hipEventRecord(b->fork, b->s0) != hipSuccess) st = fail(BD3MG_ERR_HIP, "fork record failed");
    for (size_t i = 0; i < b->probs.size() && st == BD3MG_OK; ++i) {
        if (!active[i]) continue;
        bd3mg_problem p = b->probs[i];
        if (hipStreamWaitEvent(p->stream, b->fork, 0) != hipSuccess) {
            st = fail(BD3MG_ERR_HIP, "fork wait failed");
            break;
        }
        int m[2];
        pair_modes(p, m);
        for (int sw = 0; sw < 2 && st == BD3MG_OK; ++sw) {
            for (int c = 0; c < p->ncolors && st == BD3MG_OK; ++c)
                st = phase(p, p->groups[c], false, nullptr, m[sw]);
            p->cur ^= 1;
        }
        if (st == BD3MG_OK && (hipEventRecord(b->join[i], p->stream) != hipSuccess ||
                               hipStreamWaitEvent(b->s0, b->join[i], 0) != hipSuccess))
            st = fail(BD3MG_ERR_HIP, "join failed");
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->s0, &g);
    if (st != BD3MG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(BD3MG_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
    out.graph = g;
    HIP_TRY(hipGraphInstantiate(&out.exec, out.graph, nullptr, nullptr, 0));
    out.fused = false;
    return BD3MG_OK;
}

// Whether one fused launch per pass can serve every problem: the same
// precision, z extent, in-slice radius and tile heights (template
// parameters), separable PSF, BD3MG's step, a coloured or sequential
// schedule (one source per update item).
bool batch_fusable(bd3mg_batch b)
{
    const bd3mg_problem p0 = b->probs[0];
    for (bd3mg_problem p : b->probs) {
        if (p->prec != p0->prec || p->dense || p->schedule == BD3MG_SCHED_ROUND || p->prm.method != M_BD3MG ||
            p->prm.tv3d)
            return false;
        if (p->kz != p0->kz || p->geom.R != p0->geom.R || p->geom.ty_dirs != p0->geom.ty_dirs ||
            p->geom.ty_update != p0->geom.ty_update)
            return false;
    }
    return b->probs.size() <= 255;
}

// Whether the batch runs fused launches in its mode (see bd3mg_batch_set_mode).
bool batch_uses_fused(bd3mg_batch b)
{
    if (b->mode == BD3MG_BATCH_BRANCHES || !batch_fusable(b)) return false;
    if (b->mode == BD3MG_BATCH_FUSED) return true;
    double bytes = 0.0;
    for (bd3mg_problem p : b->probs) bytes += (double)p->N * p->esz;
    return bytes <= 64.0 * 1024 * 1024;
}

// Capture two sweeps of every active problem as fused launches on the batch
// stream: for each sweep, colour index and pass, one launch whose grid holds
// the workgroups of that pass of every active problem with that colour.
template <typename T>
bd3mg_status batch_capture_fused_t(bd3mg_batch b, const std::vector<char> &active, bd3mg_batch_s::Graph &out)
{
    const int n = (int)b->probs.size();
    int maxc = 0;
    std::vector<int> modes(2 * n, 0);
    for (int i = 0; i < n; ++i)
        if (active[i]) {
            maxc = std::max(maxc, b->probs[i]->ncolors);
            pair_modes(b->probs[i], &modes[2 * i]);
        }
    struct Set {
        size_t fa0, ow0;
        unsigned nwg;
        int pass;
        bool one;
    };
    std::vector<Set> sets;
    std::vector<FusedArgs<T>> fa;
    std::vector<unsigned char> owner;
    // the direction pass runs in two launches when some problems blur d1 only
    // (H dp kept) and others both directions in the same sweep
    for (int sw = 0; sw < 2; ++sw)
        for (int c = 0; c < maxc; ++c)
            for (int pass = FP_GRAD; pass <= FP_UPDATE; ++pass)
                for (int one = 0; one < (pass == FP_DIRS ? 2 : 1); ++one) {
                Set st{fa.size(), owner.size(), 0, pass, one != 0};
                unsigned wg = 0;
                int local = 0;
                for (int i = 0; i < n; ++i) {
                    bd3mg_problem p = b->probs[i];
                    if (!active[i] || c >= p->ncolors) continue;
                    const int hm = modes[2 * i + sw];
                    if (pass == FP_DIRS && (hm == 2) != (one != 0)) continue;
                    const auto &gr = p->groups[c];
                    const int cur = p->cur;
                    p->cur = cur ^ sw;  // the previous-step buffers of this sweep
                    FusedArgs<T> a{};
                    a.g = p->geom;
                    a.prm = p->prm;
                    a.s = dev_state<T>(p);
                    hdp_state<T>(p, a.s, gr, hm);
                    p->cur = cur;
                    a.pg = p->d_pg;
                    a.pd = p->d_pd;
                    a.u = p->d_u;
                    a.info = p->d_info;
                    a.gx = (unsigned)p->geom.ntx;
                    if (pass == FP_GRAD) {
                        a.items = p->d_items + gr.g_off;
                        a.nitems = gr.g_cnt;
                        a.gy = (unsigned)p->geom.nty;
                    } else if (pass == FP_DIRS) {
                        a.items = p->d_units + gr.du_off;
                        a.nitems = gr.du_cnt;
                        a.gy = (unsigned)((p->ny + p->geom.ty_dirs - 1) / p->geom.ty_dirs);
                    } else if (pass == FP_SOLVE) {
                        a.brs = p->d_br + gr.br_off;
                        a.nitems = gr.br_cnt;
                        a.gx = a.gy = 1;
                        a.ntg = p->ntiles;
                        a.ntd = tiles_of(p->geom, p->geom.ty_dirs);
                    } else {
                        a.items = p->d_items + gr.u_off;
                        a.nitems = gr.u_cnt;
                        a.gy = (unsigned)((p->ny + p->geom.ty_update - 1) / p->geom.ty_update);
                        a.pairs = p->d_pairs;
                    }
                    a.wg0 = wg;
                    const unsigned cnt = a.gx * a.gy * (unsigned)a.nitems;
                    const unsigned end = (wg + cnt + 7) / 8 * 8;
                    for (unsigned h = wg; h < end; h += 8) owner.push_back((unsigned char)local);
                    wg = end;
                    fa.push_back(a);
                    ++local;
                }
                st.nwg = wg;
                if (wg > 0) sets.push_back(st);
                }
    if (fa.empty()) return fail(BD3MG_ERR_STATE, "no active problem in the batch");
    if (hipMalloc(&out.d_fa, fa.size() * sizeof(FusedArgs<T>)) != hipSuccess ||
        hipMalloc((void **)&out.d_owner, std::max<size_t>(owner.size(), 1)) != hipSuccess)
        return fail(BD3MG_ERR_NOMEM, "fused launch arguments");
    HIP_TRY(hipMemcpy(out.d_fa, fa.data(), fa.size() * sizeof(FusedArgs<T>), hipMemcpyHostToDevice));
    if (!owner.empty()) HIP_TRY(hipMemcpy(out.d_owner, owner.data(), owner.size(), hipMemcpyHostToDevice));
    // the problems' earlier work (set-up, checks) is complete before the graph runs
    for (bd3mg_problem p : b->probs) HIP_TRY(hipStreamSynchronize(p->stream));
    const Geom &g0 = b->probs[0]->geom;
    HIP_TRY(hipStreamBeginCapture(b->s0, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    for (const Set &st : sets) {
        if (e != hipSuccess) break;
        e = launch_fused<T>(st.pass, g0, (const FusedArgs<T> *)out.d_fa + st.fa0, out.d_owner + st.ow0, st.nwg,
                            b->s0, st.one);
    }
    hipGraph_t gph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->s0, &gph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (gph) (void)hipGraphDestroy(gph);
        return fail(BD3MG_ERR_HIP, "fused graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    out.graph = gph;
    HIP_TRY(hipGraphInstantiate(&out.exec, out.graph, nullptr, nullptr, 0));
    out.fused = true;
    return BD3MG_OK;
}

// The graph of the batch's next two sweeps in its current state: a kept one,
// or captured now (the least recently used of four dropped to make room).
bd3mg_status batch_graph(bd3mg_batch b, const std::vector<char> &active, hipGraphExec_t *exec)
{
    const std::vector<int> key = graph_key(b, active);
    for (auto &g : b->graphs)
        if (g.key == key) {
            g.used = ++b->tick;
            *exec = g.exec;
            return BD3MG_OK;
        }
    if (b->graphs.size() >= 4) {
        size_t lru = 0;
        for (size_t i = 1; i < b->graphs.size(); ++i)
            if (b->graphs[i].used < b->graphs[lru].used) lru = i;
        graph_free(b->graphs[lru]);
        b->graphs.erase(b->graphs.begin() + (long)lru);
    }
    bd3mg_batch_s::Graph g;
    bd3mg_status st;
    if (batch_uses_fused(b))
        st = b->probs[0]->prec == BD3MG_FP64 ? batch_capture_fused_t<double>(b, active, g)
                                             : batch_capture_fused_t<float>(b, active, g);
    else
        st = batch_capture(b, active, g);
    if (st != BD3MG_OK) {
        graph_free(g);
        return st;
    }
    g.key = key;
    g.used = ++b->tick;
    b->graphs.push_back(g);
    *exec = g.exec;
    return BD3MG_OK;
}

}  // namespace

extern "C" {

bd3mg_status bd3mg_batch_set_mode(bd3mg_batch b, int mode, int *fused)
{
    if (!b) return fail(BD3MG_ERR_ARG, "null batch");
    if (mode != BD3MG_BATCH_AUTO && mode != BD3MG_BATCH_FUSED && mode != BD3MG_BATCH_BRANCHES)
        return fail(BD3MG_ERR_ARG, "unknown batch mode %d", mode);
    if (mode != b->mode) batch_drop_graph(b);
    b->mode = mode;
    if (fused) *fused = batch_uses_fused(b) ? 1 : 0;
    return BD3MG_OK;
}

bd3mg_status bd3mg_batch_create(int n, const bd3mg_problem *probs, bd3mg_batch *out)
{
    if (!out) return fail(BD3MG_ERR_ARG, "null output handle");
    *out = nullptr;
    if (n < 1 || !probs) return fail(BD3MG_ERR_ARG, "need n >= 1 problems");
    for (int i = 0; i < n; ++i) {
        if (!probs[i]) return fail(BD3MG_ERR_ARG, "problem %d is null", i);
        for (int j = 0; j < i; ++j)
            if (probs[j] == probs[i]) return fail(BD3MG_ERR_ARG, "problem %d repeated", i);
        ST_TRY(ensure_ready(probs[i]));
    }
    bd3mg_batch b = new (std::nothrow) bd3mg_batch_s;
    if (!b) return fail(BD3MG_ERR_NOMEM, "batch handle");
    b->probs.assign(probs, probs + n);
    b->join.assign(n, nullptr);
    bool ok = hipStreamCreateWithFlags(&b->s0, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreate(&b->ev0) == hipSuccess && hipEventCreate(&b->ev1) == hipSuccess;
    for (int i = 0; i < n && ok; ++i)
        ok = hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        bd3mg_batch_destroy(b);
        return fail(BD3MG_ERR_HIP, "batch stream or events");
    }
    *out = b;
    return BD3MG_OK;
}

bd3mg_status bd3mg_batch_destroy(bd3mg_batch b)
{
    if (!b) return BD3MG_OK;
    if (b->s0) (void)hipStreamSynchronize(b->s0);
    batch_drop_graph(b);
    for (hipEvent_t e : b->join)
        if (e) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->s0) (void)hipStreamDestroy(b->s0);
    delete b;
    return BD3MG_OK;
}

bd3mg_status bd3mg_batch_tune(bd3mg_batch b)
{
    if (!b) return fail(BD3MG_ERR_ARG, "null batch");
    if (b->mode != BD3MG_BATCH_BRANCHES && batch_fusable(b) &&
        (b->mode == BD3MG_BATCH_FUSED || batch_uses_fused(b))) {
        // fused launches need one set of tile heights: the largest problem's
        bd3mg_problem big = b->probs[0];
        for (bd3mg_problem p : b->probs)
            if (p->N > big->N) big = p;
        int ch[2] = {0, 0};
        ST_TRY(bd3mg_autotune(big, 3, ch, nullptr));
        for (bd3mg_problem p : b->probs)
            if (p->prec == big->prec && !p->dense) {
                p->geom.ty_dirs = ch[0];
                p->geom.ty_update = ch[1];
            }
    } else {
        for (bd3mg_problem p : b->probs) ST_TRY(bd3mg_autotune(p, 3, nullptr, nullptr));
    }
    batch_drop_graph(b);  // tile heights are baked into the captured launches
    return BD3MG_OK;
}

bd3mg_status bd3mg_batch_run(bd3mg_batch b, int max_sweeps, double grad_rtol, int check_every,
                             bd3mg_result *results)
{
    if (!b) return fail(BD3MG_ERR_ARG, "null batch");
    if (max_sweeps < 0 || check_every < 0) return fail(BD3MG_ERR_ARG, "negative sweep count");
    const int n = (int)b->probs.size();
    for (bd3mg_problem p : b->probs) ST_TRY(ensure_ready(p));
    const bool stopping = grad_rtol > 0.0;
    int ce = check_every > 0 ? check_every : 16;
    ce += ce & 1;  // checks fall between graph launches of two sweeps
    std::vector<char> active(n, 1), conv(n, 0);
    std::vector<int> done(n, 0);
    HIP_TRY(hipEventRecord(b->ev0, b->s0));
    int s = 0;
    auto sync_all = [&]() -> bd3mg_status {
        HIP_TRY(hipStreamSynchronize(b->s0));
        return BD3MG_OK;
    };
    for (; s + 2 <= max_sweeps; s += 2) {
        bool any = false;
        for (int i = 0; i < n; ++i) any = any || active[i];
        if (!any) break;
        hipGraphExec_t exec = nullptr;
        ST_TRY(batch_graph(b, active, &exec));
        HIP_TRY(hipGraphLaunch(exec, b->s0));
        bool need_sync = stopping && ((s + 2) % ce == 0);
        for (int i = 0; i < n; ++i) {
            if (!active[i]) continue;
            bd3mg_problem p = b->probs[i];
            int m[2];
            pair_modes(p, m);
            p->hdp_valid = m[1] != 0;
            done[i] += 2;
            p->sweeps_done += 2;
            if (p->refresh_every > 0 && p->sweeps_done / p->refresh_every != (p->sweeps_done - 2) / p->refresh_every)
                need_sync = true;
        }
        if (!need_sync) continue;
        ST_TRY(sync_all());
        for (int i = 0; i < n; ++i) {
            if (!active[i]) continue;
            bd3mg_problem p = b->probs[i];
            if (p->refresh_every > 0 && p->sweeps_done / p->refresh_every != (p->sweeps_done - 2) / p->refresh_every)
                ST_TRY(refresh(p, p->x, p->q));
            if (stopping && (s + 2) % ce == 0) {
                double gn = 0.0;
                ST_TRY(eval_at(p, p->x, p->q, nullptr, &gn));
                if (gn <= grad_rtol * p->gnorm_ref) {
                    // confirmed on a residual rebuilt from x (as bd3mg_run does)
                    ST_TRY(ensure_tmp(p, 2));
                    ST_TRY(refresh(p, p->x, p->tmp[1]));
                    ST_TRY(eval_at(p, p->x, p->tmp[1], nullptr, &gn));
                }
                if (gn <= grad_rtol * p->gnorm_ref) {
                    conv[i] = 1;
                    active[i] = 0;
                }
            }
        }
        for (int i = 0; i < n; ++i) HIP_TRY(hipStreamSynchronize(b->probs[i]->stream));
    }
    ST_TRY(sync_all());
    if (s < max_sweeps) {  // one more sweep, launched directly
        for (int i = 0; i < n; ++i) {
            if (!active[i]) continue;
            bd3mg_problem p = b->probs[i];
            const int hm = hdp_mode(p, false, p->sweeps_done, p->hdp_valid);
            for (int c = 0; c < p->ncolors; ++c) ST_TRY(phase(p, p->groups[c], false, nullptr, hm));
            p->hdp_valid = hm != 0;
            p->cur ^= 1;
            done[i] += 1;
            p->sweeps_done += 1;
        }
    }
    HIP_TRY(hipEventRecord(b->ev1, b->s0));
    for (int i = 0; i < n; ++i) HIP_TRY(hipStreamSynchronize(b->probs[i]->stream));
    HIP_TRY(hipEventSynchronize(b->ev1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    bool all = true;
    for (int i = 0; i < n; ++i) {
        bd3mg_problem p = b->probs[i];
        double f = 0.0, gn = 0.0;
        ST_TRY(ensure_tmp(p, 2));
        ST_TRY(refresh(p, p->x, p->tmp[1]));
        ST_TRY(eval_at(p, p->x, p->tmp[1], &f, &gn));
        if (stopping && !conv[i] && gn <= grad_rtol * p->gnorm_ref) conv[i] = 1;
        all = all && (conv[i] || !stopping);
        if (results) {
            results[i].sweeps = done[i];
            results[i].converged = conv[i];
            results[i].f = f;
            results[i].grad_norm = gn;
            results[i].grad_norm_ref = p->gnorm_ref;
            results[i].seconds = ms * 1e-3;
        }
    }
    if (!all) return fail(BD3MG_ERR_NOT_CONVERGED, "some problems of the batch did not converge");
    return BD3MG_OK;
}

}  // extern "C"
