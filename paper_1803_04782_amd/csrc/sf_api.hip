// C-ABI layer of libsf: scene object, validation, device memory, tick loop.
// The declarations and their contracts are in include/sf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "sf.h"
#include "sf_internal.h"

using sf::FieldLaunch;
using sf::ListCfg;
using sf::SceneView;
using sf::SupCfg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return fail(SF_ENOMEM, "%s: out of device memory", what);
    return fail(SF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SF_HIP(call, what)                            \
    do {                                              \
        const hipError_t e_ = (call);                 \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

struct sf_scene {
    // description
    int W = 0, H = 0, N = 0, R = 0, R_obs = 0;
    int fp = 0;  // row pitch of S, P, phi and phi32 (sf::field_pitch(W))
    double k = 1, alpha = -0.5, k_obs = 1, alpha_obs = -0.5, w_dest = 1;
    unsigned long long seed = 0;
    int64_t start_step = 0;
    bool periodic = false;
    double w_heading = 1;
    std::vector<uint8_t> h_heading;  // by caller id; empty: no headings
    std::vector<uint8_t> h_walk;     // walk periods by caller id; empty: none
    int bw = 1, bh = 1;              // body width and height (odd)
    int device = 0;
    hipStream_t stream = nullptr;
    int ncu = 0;
    // layout
    int wpr = 0;          // 64-bit words per bitmap row
    ListCfg lc;           // pedestrian field launch shape
    float phi_axial = 0.f, phi_diag = 0.f;
    // device state: S = w_dest*D + O (FP64), P = fl32(S + Phi), the stamp as
    // doubles and (laws that allow 32-bit sums, see law_units) as integers in
    // units of q
    double *S = nullptr, *tab = nullptr;
    int32_t *tabi = nullptr;
    double q_unit = 1.0;
    bool int_ok = false;
    int int_rounds = 1;  // rounds of 8 integer terms summed in 32 bits (see law_units)
    float *P = nullptr;
    int32_t *D = nullptr;
    uint8_t *exitm = nullptr;
    unsigned long long *occ = nullptr, *key = nullptr;
    sf::ClaimRec *claims = nullptr;  // per su: election word and registration count
    int32_t *pos = nullptr, *target = nullptr;
    // Per-pedestrian arrays use internal ids: live pedestrians in row-major
    // order of their positions when the state was set, then the evacuated
    // ones, so that neighbouring su hold neighbouring ids.  ext (device) and
    // h_ext (host) map an internal id to the caller's id.
    int32_t *ext = nullptr;
    std::vector<int32_t> h_ext;
    uint8_t *heading = nullptr;  // by internal id (NULL: no headings)
    uint8_t *walk = nullptr;     // walk periods by internal id (NULL: none)
    uint8_t *flags = nullptr;
    unsigned long long *ctr = nullptr;  // see sf::ctr_index
    // what the per-tick kernels read: the view (host copy and device copy),
    // the field work items and the launch sizes
    SceneView view = {};
    int strips_per_block = 1;  // field: strips per work item (items dealt round robin)
    // single-scene field launches use the dense small-radius stencil (same
    // result bit for bit as the gather, which batches keep using)
    bool dense = false;
    // incremental field update (sf_set_field_update): refresh period, ticks
    // since the last full superposition, the moved bitmaps and the update
    // view (S = P, sources = the su entered, moved_from = the su left)
    int refresh = 0, since_full = 0;
    unsigned long long *moved_from = nullptr, *moved_to = nullptr;
    double *phi = nullptr;  // exact pedestrian field (FP64) kept for the updates
    // bodies larger than one su: covered su and (bounded grids) obstacles
    unsigned long long *bodies = nullptr, *obits = nullptr;
    // the paper's own field path (sf_set_field_sect): K slots (0 = off), the
    // term list, the kept FP32 field and the optional 8-plane sect image
    int sect_K = 0;
    bool sect_image = false;
    int2 *sect_terms = nullptr;
    float *phi32 = nullptr, *image = nullptr;
    sf::SectView sect_view = {};
    SceneView view_upd = {};
    FieldLaunch fl;
    // batch membership: while a batch holds the scene, `stream` is the
    // batch's stream and `own_stream` the one given at create
    sf_batch *batch = nullptr;
    hipStream_t own_stream = nullptr;
    std::vector<void *> owned;
    // timing
    bool timing = false;
    std::vector<EventPair> ev[SF_KERNEL_COUNT];
    size_t ev_used[SF_KERNEL_COUNT] = {};
};

namespace {

// Device-side layout of one group of a batch for one tiling: the member
// views, the workgroup -> scene maps of the decide and commit launches, the
// field work items and the stamp tables (one per distinct radius and law).
struct GroupLayout {
    sf_group_tiling t = {};
    std::vector<int> members;  // indices into sf_batch::scenes
    FieldLaunch fl;
    int n_items = 0, dec_blocks = 0, com_blocks = 0;
    SceneView *d_views = nullptr;
    int32_t *d_dec_scene = nullptr, *d_com_scene = nullptr, *d_items = nullptr;
    unsigned int *d_queue = nullptr;  // the field launch's work-queue counters (zero between launches)
    std::vector<void *> bufs;
};

struct BatchLayout {
    sf_batch_tiling t = {};
    int n_groups = 0;
    GroupLayout g[SF_MAX_GROUPS];
    SceneView *d_all = nullptr;               // every member, batch order (totals)
    unsigned long long *d_totals = nullptr;   // 16 words per scene (sf_batch_stats)
    std::vector<void *> bufs;
};

}  // namespace

struct sf_batch {
    int device = 0;
    hipStream_t stream = nullptr;   // where ticks run (caller's stream)
    // ticks of groups 1.. (forked from and joined back to `stream`)
    hipStream_t aux[SF_MAX_GROUPS - 1] = {};
    hipStream_t capture = nullptr;  // private streams on which graphs are captured
    hipStream_t capture_aux[SF_MAX_GROUPS - 1] = {};
    hipEvent_t fork = nullptr, join[SF_MAX_GROUPS - 1] = {};
    int ncu = 0;
    size_t max_lds = 0;
    std::vector<sf_scene *> scenes;
    bool broken = false;  // a member scene was destroyed
    BatchLayout cur;
    // captured graphs by ticks per replay
    std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
};

namespace {

template <typename T>
int dalloc(sf_scene *s, T **p, size_t n, const char *what)
{
    void *q = nullptr;
    const size_t bytes = (n ? n : 1) * sizeof(T);
    const hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return hip_fail(e, what);
    s->owned.push_back(q);
    *p = static_cast<T *>(q);
    return SF_OK;
}

void release(sf_scene *s)
{
    if (!s) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (sf_batch *b = s->batch) {
        // the batch can no longer run: its views name this scene's memory
        b->broken = true;
        b->scenes.erase(std::remove(b->scenes.begin(), b->scenes.end(), s), b->scenes.end());
    }
    for (void *p : s->owned) (void)hipFree(p);
    for (int k = 0; k < SF_KERNEL_COUNT; ++k)
        for (EventPair &e : s->ev[k]) {
            if (e.a) (void)hipEventDestroy(e.a);
            if (e.b) (void)hipEventDestroy(e.b);
        }
    (void)hipSetDevice(cur);
    delete s;
}

// Scoped switch to the scene's device.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else if (prev == dev) prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Stamp of the law phi(d) = k*|d|_2^alpha on the window |d|_inf <= R (zero at
// d = 0 and outside it), each strength rounded once to FP32 and held as a
// double: entry (dx, dy) at (dx + padx)*stride + dy + pady of a column-major
// table of n doubles with ncols columns of nrows rows around row pady, zero
// elsewhere (the nonzero band |dy| <= R lies inside each column's stride).
std::vector<double> stamp_table(int R, double k, double alpha, int ncols, int nrows, int stride,
                                int padx, int pady, size_t n)
{
    std::vector<double> t(n, 0.0);
    for (int ci = 0; ci < ncols; ++ci)
        for (int ri = std::max(0, pady - R); ri < nrows && ri <= pady + R; ++ri) {
            const int dx = ci - padx, dy = ri - pady;
            if (std::abs(dx) > R || std::abs(dy) > R || (dx == 0 && dy == 0)) continue;
            if (ri >= stride || (size_t)ci * stride + ri >= n) continue;  // not reached
            const double dist = std::sqrt((double)dx * dx + (double)dy * dy);
            t[(size_t)ci * stride + ri] = (double)(float)(k * std::pow(dist, alpha));
        }
    return t;
}

// Copy a host table to the device and wait for the copy.
int upload_table(double *dst, const std::vector<double> &t, hipStream_t st)
{
    SF_HIP(hipMemcpyAsync(dst, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, st),
           "copy stamp");
    SF_HIP(hipStreamSynchronize(st), "stamp sync");
    return SF_OK;
}

// The gather's integer form of a law (sf::ListCfg elem = 4): every FP32
// strength of the window is an integer multiple of q = 2^(e_min - 23), e_min
// the exponent of the smallest nonzero |strength| (the same q as check_law),
// and the kernel sums 8 of them in a 32-bit integer before moving the sum into
// FP64, which needs 8 * max|strength| / q < 2^31.
// The gather may sum `rounds` rounds of 8 terms in 32 bits when
// 8 * rounds * max|strength| / q < 2^31 (at most 64 rounds).
struct LawUnits {
    double q = 1.0;
    bool int_ok = true;
    int rounds = 1;
};

LawUnits law_units(int R, double k, double alpha)
{
    double tmin = 0.0, tmax = 0.0;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const double dist = std::sqrt((double)dx * dx + (double)dy * dy);
            const double a = std::fabs((double)(float)(k * std::pow(dist, alpha)));
            if (a == 0.0) continue;
            tmin = tmin == 0.0 || a < tmin ? a : tmin;
            tmax = a > tmax ? a : tmax;
        }
    LawUnits u;
    if (tmax == 0.0) return u;
    int e;
    (void)std::frexp(tmin, &e);
    u.q = std::ldexp(1.0, std::max(e - 1 - 23, -149));
    u.int_ok = 8.0 * (tmax / u.q) < 2147483648.0;
    if (u.int_ok)
        u.rounds = (int)std::min(64.0, std::floor(2147483647.0 / (8.0 * (tmax / u.q))));
    return u;
}

// The stamp of stamp_table in units of q (exact integers).
std::vector<int32_t> stamp_table_int(const std::vector<double> &t, double q)
{
    std::vector<int32_t> r(t.size());
    for (size_t i = 0; i < t.size(); ++i) r[i] = (int32_t)(t[i] / q);
    return r;
}

// The superposition adds FP32 strengths in FP64.  Every term of a window is
// an integer multiple of q = 2^(e_min - 23), e_min the exponent of the
// smallest nonzero |strength|, and every partial sum of one su's terms (each
// window offset at most once, or up to twice for the incremental update's
// previous field plus the entered sources) is bounded by 2*sum|strength|.
// When 4*sum|strength| < 2^53 * q every such sum is an FP64 number, so the
// field does not depend on the order of its terms.  Laws outside that range
// (strengths spread over more than about 2^15 within one window) are refused.
int check_law(int R, double k, double alpha, const char *what)
{
    double sum = 0.0, tmin = 0.0;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const double dist = std::sqrt((double)dx * dx + (double)dy * dy);
            const float t = (float)(k * std::pow(dist, alpha));
            if (!std::isfinite(t))
                return fail(SF_EINVAL, "%s law k = %g, alpha = %g: strength at (%d, %d) is not "
                            "a finite FP32 number", what, k, alpha, dx, dy);
            const double a = std::fabs((double)t);
            if (a == 0.0) continue;
            sum += a;
            tmin = tmin == 0.0 || a < tmin ? a : tmin;
        }
    if (sum == 0.0) return SF_OK;
    int e;
    (void)std::frexp(tmin, &e);  // tmin = f * 2^e, f in [0.5, 1): exponent e - 1
    const double q = std::ldexp(1.0, std::max(e - 1 - 23, -149));
    if (4.0 * sum >= std::ldexp(q, 53))
        return fail(SF_EINVAL, "%s law k = %g, alpha = %g, radius %d: strengths from %g to a "
                    "window sum of %g are too far apart for exact FP64 sums", what, k, alpha, R,
                    tmin, sum);
    return SF_OK;
}

// Persistent workgroups per compute unit of a single-scene field launch: as
// many as a compute unit holds at once (LDS, registers, 32 waves); more would
// run as a partial second round.
int field_blocks_per_cu(const ListCfg &lc)
{
    int per_cu = (int)std::max<size_t>(1, (size_t)(160 * 1024) / lc.lds_bytes);
    per_cu = std::min(per_cu, std::max(1, 32 / lc.nw));
    const int resident =
        sf::field_resident_blocks(lc.tw, lc.hl, lc.nw, lc.lds_bytes, false, lc.elem, lc.vec);
    if (resident > 0) per_cu = std::min(per_cu, resident);
    return per_cu;
}

int validate(const sf_scene_desc *d)
{
    if (!d) return fail(SF_EINVAL, "descriptor is NULL");
    if (d->width <= 0 || d->height <= 0)
        return fail(SF_EINVAL, "grid %d x %d: both sides must be positive", d->width, d->height);
    if ((int64_t)d->width * d->height >= (int64_t)1 << 31)
        return fail(SF_EINVAL, "grid %d x %d has 2^31 su or more", d->width, d->height);
    if (!d->obstacle || !d->exit) return fail(SF_EINVAL, "obstacle and exit masks are required");
    if (d->n_peds < 0) return fail(SF_EINVAL, "n_peds = %d is negative", d->n_peds);
    if (d->n_peds > SF_MAX_PEDS)
        return fail(SF_EINVAL, "n_peds = %d is above %d", d->n_peds, SF_MAX_PEDS);
    if (d->n_peds > 0 && !d->pos) return fail(SF_EINVAL, "pos is NULL with n_peds = %d", d->n_peds);
    if (d->radius < 0 || d->radius > SF_MAX_RADIUS)
        return fail(SF_EINVAL, "radius %d outside 0..%d", d->radius, SF_MAX_RADIUS);
    if (d->radius_obs < -1 || d->radius_obs > SF_MAX_RADIUS)
        return fail(SF_EINVAL, "radius_obs %d outside -1..%d", d->radius_obs, SF_MAX_RADIUS);
    const double params[6] = {d->k, d->alpha, d->k_obs, d->alpha_obs, d->w_dest, d->w_heading};
    for (double v : params)
        if (!std::isfinite(v)) return fail(SF_EINVAL, "field parameters must be finite");
    if (d->start_step < 0) return fail(SF_EINVAL, "start_step %lld is negative",
                                       (long long)d->start_step);
    {
        int rc = check_law(d->radius, d->k, d->alpha, "pedestrian");
        if (rc) return rc;
        if (!d->periodic &&
            (rc = check_law(d->radius_obs < 0 ? d->radius : d->radius_obs, d->k_obs,
                            d->alpha_obs, "obstacle")))
            return rc;
    }
    if (d->periodic != 0 && d->periodic != 1)
        return fail(SF_EINVAL, "periodic = %d is neither 0 nor 1", d->periodic);
    if (d->heading)
        for (int i = 0; i < d->n_peds; ++i)
            if (d->heading[i] > 8)
                return fail(SF_EINVAL, "pedestrian %d has heading %d above 8", i, d->heading[i]);
    if (d->walk_period)
        for (int i = 0; i < d->n_peds; ++i)
            if (d->walk_period[i] == 0)
                return fail(SF_EINVAL, "pedestrian %d has walk period 0", i);
    const int bw = d->body_w ? d->body_w : 1, bh = d->body_h ? d->body_h : 1;
    if (bw < 1 || bh < 1 || bw > SF_MAX_BODY || bh > SF_MAX_BODY || !(bw & 1) || !(bh & 1))
        return fail(SF_EINVAL, "body %d x %d: sides must be odd, 1..%d", bw, bh, SF_MAX_BODY);
    if (bw > d->width || bh > d->height)
        return fail(SF_EINVAL, "body %d x %d is larger than the grid", bw, bh);
    const int64_t n = (int64_t)d->width * d->height;
    if (d->periodic) {
        // a torus: the halo words of the field kernel wrap at most once
        if (d->width < 64)
            return fail(SF_EINVAL, "periodic grid width %d is below 64", d->width);
        if (2 * d->radius + 1 > std::min(d->width, d->height))
            return fail(SF_EINVAL, "periodic grid %d x %d is narrower than the %d-su window",
                        d->width, d->height, 2 * d->radius + 1);
        for (int64_t c = 0; c < n; ++c)
            if (d->obstacle[c] || d->exit[c])
                return fail(SF_EINVAL, "periodic scene has an obstacle or exit at su %lld",
                            (long long)c);
        return SF_OK;
    }
    int64_t exits = 0;
    for (int64_t c = 0; c < n; ++c) {
        if (d->exit[c]) {
            if (d->obstacle[c])
                return fail(SF_EINVAL, "su %lld is both exit and obstacle", (long long)c);
            ++exits;
        }
    }
    if (exits == 0) return fail(SF_EINVAL, "the scene has no exit su");
    return SF_OK;
}

// Pedestrian positions must be in range and their bodies (half-widths a, b;
// 0, 0 = one su) inside the grid (or wrapped on a torus), on free non-exit su
// and disjoint (evacuated = -1 allowed when `allow_gone`).
int validate_positions(int W, int H, const uint8_t *obst, const uint8_t *exitm, int N,
                       const int32_t *pos, bool allow_gone, int a = 0, int b = 0,
                       bool periodic = false)
{
    const int64_t n = (int64_t)W * H;
    std::vector<uint64_t> seen((size_t)(n + 63) / 64, 0);
    for (int i = 0; i < N; ++i) {
        const int32_t p = pos[i];
        if (p == -1 && allow_gone) continue;
        if (p < 0 || p >= n) return fail(SF_EINVAL, "pedestrian %d at su %d is outside the grid", i, p);
        const int x = p % W, y = p / W;
        for (int j = -b; j <= b; ++j)
            for (int k = -a; k <= a; ++k) {
                int sx = x + k, sy = y + j;
                if (periodic) {
                    sx = (sx % W + W) % W;
                    sy = (sy % H + H) % H;
                } else if (sx < 0 || sy < 0 || sx >= W || sy >= H) {
                    return fail(SF_EINVAL, "the body of pedestrian %d at su %d leaves the grid",
                                i, p);
                }
                const int64_t c = (int64_t)sy * W + sx;
                if (obst[c]) return fail(SF_EINVAL, "pedestrian %d covers obstacle su %lld", i,
                                         (long long)c);
                if (exitm[c]) return fail(SF_EINVAL, "pedestrian %d covers exit su %lld", i,
                                          (long long)c);
                uint64_t &w = seen[(size_t)c >> 6];
                const uint64_t bit = 1ull << (c & 63);
                if (w & bit) return fail(SF_EINVAL, "pedestrian %d shares su %lld with another",
                                         i, (long long)c);
                w |= bit;
            }
    }
    return SF_OK;
}

// Event pair that the next launch of kernel k records (nullptr when not timing).
int timing_events(sf_scene *s, int k, sf::LaunchEvents *ev)
{
    ev->start = ev->stop = nullptr;
    if (!s->timing) return SF_OK;
    if (s->ev_used[k] == s->ev[k].size()) {
        EventPair e;
        // no system-scope fence: the timestamps are only read back by this library
        SF_HIP(hipEventCreateWithFlags(&e.a, hipEventDisableSystemFence), "hipEventCreate");
        SF_HIP(hipEventCreateWithFlags(&e.b, hipEventDisableSystemFence), "hipEventCreate");
        s->ev[k].push_back(e);
    }
    ev->start = s->ev[k][s->ev_used[k]].a;
    ev->stop = s->ev[k][s->ev_used[k]].b;
    ++s->ev_used[k];
    return SF_OK;
}

// One single-scene field launch with view `v` (the scene's own, or an update view).
hipError_t scene_field(const sf_scene *s, const SceneView &v, hipStream_t st,
                       const sf::LaunchEvents *ev = nullptr)
{
    if (s->sect_K)
        return sf::launch_field_sect(s->sect_view, s->ncu * 8, false, s->sect_image, st, ev);
    if (s->dense) return sf::launch_field_dense(v, s->ncu * 8, st, ev);
    return sf::launch_field_one(s->fl, v, s->strips_per_block, st, ev);
}

// Occupancy and live count from the current positions, then the
// field of those positions.  Other counters are left as they are.
int rebuild_dynamic(sf_scene *s)
{
    s->since_full = 0;
    if (s->moved_from) {
        const size_t nwords = (size_t)s->wpr * s->H;
        SF_HIP(sf::launch_fill_u64(s->moved_from, nwords, 0ull, s->stream), "clear moves");
        SF_HIP(sf::launch_fill_u64(s->moved_to, nwords, 0ull, s->stream), "clear moves");
    }
    const size_t nwords = (size_t)s->wpr * s->H;
    SF_HIP(sf::launch_fill_u64(s->occ, nwords, 0ull, s->stream), "clear occupancy");
    SF_HIP(sf::launch_occ_init(s->pos, s->N, s->occ, s->wpr, s->W, s->ctr, s->stream),
           "occupancy");
    if (s->bodies) {
        SF_HIP(sf::launch_fill_u64(s->bodies, nwords, 0ull, s->stream), "clear bodies");
        SF_HIP(sf::launch_body_init(s->view, s->stream), "bodies");
    }
    SF_HIP(scene_field(s, s->view, s->stream), "superpose");
    return SF_OK;
}

// Zero all running totals and set the tick index.
int reset_counters(sf_scene *s, int64_t step, int64_t evacuated)
{
    SF_HIP(sf::launch_fill_u64(s->ctr, sf::kCtrWords, 0ull, s->stream), "clear counters");
    SF_HIP(sf::launch_fill_u64(s->ctr, 1, (unsigned long long)step, s->stream), "step");
    SF_HIP(sf::launch_fill_u64(s->ctr + sf::ctr_index(sf::kEvacuated, 0), 1,
                               (unsigned long long)evacuated, s->stream),
           "evacuated");
    return SF_OK;
}

int64_t counter_sum(const unsigned long long *h, int id)
{
    unsigned long long v = 0;
    for (int k = 0; k < sf::kSlots; ++k) v += h[sf::ctr_index(id, k)];
    return (int64_t)v;
}

int64_t counter_max(const unsigned long long *h, int id)
{
    unsigned long long v = 0;
    for (int k = 0; k < sf::kSlots; ++k) v = std::max(v, h[sf::ctr_index(id, k)]);
    return (int64_t)v;
}

int build_statics(sf_scene *s, const uint8_t *h_obst, const uint8_t *h_exit)
{
    const int W = s->W, H = s->H, n = W * H;
    hipStream_t st = s->stream;
    if (s->periodic) {
        // a torus without obstacles or openings: no static field
        SF_HIP(sf::launch_fill_i32(s->D, (size_t)n, 0, st), "destination field");
        SF_HIP(sf::launch_fill_u64(reinterpret_cast<unsigned long long *>(s->S),
                                   (size_t)s->fp * H, 0ull, st),
               "static field");
        SF_HIP(hipMemcpyAsync(s->exitm, h_exit, (size_t)n, hipMemcpyHostToDevice, st),
               "copy exits");
        SF_HIP(hipStreamSynchronize(st), "statics sync");
        return SF_OK;
    }
    uint8_t *obst = nullptr;
    unsigned int *active = nullptr;
    unsigned long long *obits = nullptr, *vis[2] = {nullptr, nullptr},
                       *front[2] = {nullptr, nullptr};
    double *tab64 = nullptr, *O = nullptr;
    int rc;
    // temporaries are released right after the statics are built
    const size_t first_tmp = s->owned.size();
    const size_t nbw = (size_t)s->wpr * H;
    if ((rc = dalloc(s, &obst, (size_t)n, "obstacle mask")) ||
        (rc = dalloc(s, &obits, nbw, "obstacle bitmap")) ||
        (rc = dalloc(s, &vis[0], nbw, "BFS visited set")) ||
        (rc = dalloc(s, &vis[1], nbw, "BFS visited set")) ||
        (rc = dalloc(s, &front[0], nbw, "BFS frontier")) ||
        (rc = dalloc(s, &front[1], nbw, "BFS frontier")) ||
        (rc = dalloc(s, &active, (size_t)sf::bfs_ring(), "BFS counters")))
        return rc;
    SF_HIP(hipMemcpyAsync(obst, h_obst, (size_t)n, hipMemcpyHostToDevice, st), "copy obstacles");
    SF_HIP(hipMemcpyAsync(s->exitm, h_exit, (size_t)n, hipMemcpyHostToDevice, st), "copy exits");
    SF_HIP(sf::launch_mask_to_bits(obst, obits, W, H, s->wpr, st), "obstacle bitmap");
    if (s->obits)  // kept for the move tests of bodies larger than one su
        SF_HIP(hipMemcpyAsync(s->obits, obits, nbw * sizeof(unsigned long long),
                              hipMemcpyDeviceToDevice, st),
               "keep obstacle bitmap");

    // destination field: BFS over free su from the exit set, a batch of
    // launches between looks at whether a frontier is left
    SF_HIP(sf::launch_bfs_seed(s->exitm, s->D, n, st), "BFS seed");
    SF_HIP(sf::launch_mask_to_bits(s->exitm, vis[0], W, H, s->wpr, st), "BFS seed");
    SF_HIP(sf::launch_mask_to_bits(s->exitm, front[0], W, H, s->wpr, st), "BFS seed");
    SF_HIP(sf::launch_fill_i32(reinterpret_cast<int32_t *>(active), sf::bfs_ring(), 0, st),
           "clear BFS counters");
    // no distance exceeds the number of su
    const long long max_launches = (long long)n / sf::bfs_levels_per_launch() + 2;
    const int per_look = 8;
    for (int j = 0;; ++j) {
        SF_HIP(sf::launch_bfs_block(obits, vis, front, s->D, W, H, s->wpr, j, active, st),
               "BFS levels");
        if ((j + 1) % per_look) continue;
        unsigned int left = 0;
        SF_HIP(hipMemcpyAsync(&left, &active[j % sf::bfs_ring()], sizeof left,
                              hipMemcpyDeviceToHost, st),
               "BFS frontier flag");
        SF_HIP(hipStreamSynchronize(st), "BFS sync");
        if (left == 0) break;
        if (j > max_launches) return fail(SF_EDEVICE, "BFS did not terminate");
    }
    SF_HIP(sf::launch_fill_u64(s->ctr, sf::kCtrWords, 0ull, st), "clear counters");
    SF_HIP(sf::launch_count_unreachable(obst, s->D, n, s->ctr, st), "reachability");
    std::vector<unsigned long long> hc(sf::kCtrWords);
    SF_HIP(hipMemcpyAsync(hc.data(), s->ctr, sf::kCtrWords * 8, hipMemcpyDeviceToHost, st),
           "reachability copy");
    SF_HIP(hipStreamSynchronize(st), "reachability sync");
    const long long unreachable = counter_sum(hc.data(), sf::kScratch);
    if (unreachable)
        return fail(SF_EUNREACHABLE, "%lld free su cannot reach any exit", unreachable);

    // obstacle field (exact FP64 sums of FP32 strengths), fused with the
    // destination field into S
    const SupCfg oc = sf::make_sup_cfg(s->R_obs, 8, 1, sizeof(double));
    SupCfg ocg = oc;
    if ((rc = dalloc(s, &tab64, (size_t)oc.ncols * oc.stride, "obstacle table")) ||
        (rc = dalloc(s, &O, (size_t)n, "obstacle field")))
        return rc;
    {
        int max_lds = 0;
        SF_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                     s->device),
               "LDS size");
        if ((size_t)max_lds < oc.lds_bytes)
            return fail(SF_EINVAL, "obstacle table needs %zu B of LDS, device has %d B",
                        oc.lds_bytes, max_lds);
        SF_HIP(sf::set_superpose_lds_limit((size_t)max_lds), "LDS limit");
        ocg.grid = std::max(1, s->ncu * (int)std::max<size_t>(1, (size_t)max_lds / oc.lds_bytes));
    }
    if ((rc = upload_table(tab64,
                           stamp_table(s->R_obs, s->k_obs, s->alpha_obs, oc.ncols, oc.nrows,
                                       oc.stride, oc.padx, oc.pady,
                                       (size_t)oc.ncols * oc.stride),
                           st)))
        return rc;
    SF_HIP(sf::launch_superpose_f64(ocg, obits, s->wpr, tab64, O, W, H, st), "obstacle field");
    // the padding columns of S are never read; they are cleared all the same
    SF_HIP(sf::launch_fill_u64(reinterpret_cast<unsigned long long *>(s->S), (size_t)s->fp * H,
                               0ull, st),
           "static field");
    SF_HIP(sf::launch_static_S(s->D, O, obst, s->w_dest, s->S, W, H, s->fp, st), "static field");
    SF_HIP(hipStreamSynchronize(st), "statics sync");
    for (size_t i = first_tmp; i < s->owned.size(); ++i) (void)hipFree(s->owned[i]);
    s->owned.resize(first_tmp);
    return SF_OK;
}

int setup_launches(sf_scene *s);

// Positions by caller id -> internal order (see sf_scene::ext), uploaded with
// the id map.  Blocks until the copies are done.
int upload_positions(sf_scene *s, const int32_t *pos)
{
    const int N = s->N;
    std::vector<int32_t> order((size_t)N), pint((size_t)N);
    // sort (position, id) pairs packed in 64-bit keys; evacuated (-1) read as
    // the largest unsigned position and go last, in id order
    std::vector<uint64_t> keyed((size_t)N);
    for (int i = 0; i < N; ++i)
        keyed[(size_t)i] = ((uint64_t)(uint32_t)pos[i] << 32) | (uint32_t)i;
    std::sort(keyed.begin(), keyed.end());
    for (int i = 0; i < N; ++i) {
        order[(size_t)i] = (int32_t)(uint32_t)keyed[(size_t)i];
        pint[(size_t)i] = (int32_t)(keyed[(size_t)i] >> 32);
    }
    s->h_ext = order;
    // per-pedestrian attributes follow the internal order
    std::vector<uint8_t> hint((size_t)N), wint((size_t)N);
    if (N && s->heading) {
        for (int i = 0; i < N; ++i) hint[(size_t)i] = s->h_heading[(size_t)order[(size_t)i]];
        SF_HIP(hipMemcpyAsync(s->heading, hint.data(), (size_t)N, hipMemcpyHostToDevice,
                              s->stream),
               "copy headings");
    }
    if (N && s->walk) {
        for (int i = 0; i < N; ++i) wint[(size_t)i] = s->h_walk[(size_t)order[(size_t)i]];
        SF_HIP(hipMemcpyAsync(s->walk, wint.data(), (size_t)N, hipMemcpyHostToDevice, s->stream),
               "copy walk periods");
    }
    if (N) {
        SF_HIP(hipMemcpyAsync(s->pos, pint.data(), (size_t)N * sizeof(int32_t),
                              hipMemcpyHostToDevice, s->stream),
               "copy positions");
        SF_HIP(hipMemcpyAsync(s->ext, order.data(), (size_t)N * sizeof(int32_t),
                              hipMemcpyHostToDevice, s->stream),
               "copy id map");
    }
    SF_HIP(hipStreamSynchronize(s->stream), "positions sync");
    return SF_OK;
}

// Copy a per-pedestrian array to caller order: dst[ext[i]] = src[i].
template <typename T>
int copy_by_caller_id(const sf_scene *s, T *dst, const T *src, int dst_on_device,
                      T mask = (T)-1)
{
    const int N = s->N;
    if (!dst || N == 0) return SF_OK;
    if (dst_on_device) {
        hipError_t e;
        if constexpr (sizeof(T) == 4)
            e = sf::launch_scatter_i32(reinterpret_cast<const int32_t *>(src), s->ext,
                                       reinterpret_cast<int32_t *>(dst), N, s->stream);
        else
            e = sf::launch_scatter_u8(reinterpret_cast<const uint8_t *>(src), s->ext,
                                      reinterpret_cast<uint8_t *>(dst), N, (uint8_t)mask,
                                      s->stream);
        SF_HIP(e, "scatter by id");
        return SF_OK;
    }
    std::vector<T> tmp((size_t)N);
    SF_HIP(hipMemcpyAsync(tmp.data(), src, (size_t)N * sizeof(T), hipMemcpyDeviceToHost, s->stream),
           "copy out");
    SF_HIP(hipStreamSynchronize(s->stream), "copy out sync");
    for (int i = 0; i < N; ++i) dst[s->h_ext[(size_t)i]] = (T)(tmp[(size_t)i] & mask);
    return SF_OK;
}

int create(const sf_scene_desc *d, void *hip_stream, sf_scene **out)
{
    int rc = validate(d);
    if (rc) return rc;
    const int bw = d->body_w ? d->body_w : 1, bh = d->body_h ? d->body_h : 1;
    if ((rc = validate_positions(d->width, d->height, d->obstacle, d->exit, d->n_peds, d->pos,
                                 false, (bw - 1) / 2, (bh - 1) / 2, d->periodic != 0)))
        return rc;
    sf_scene *s = new (std::nothrow) sf_scene;
    if (!s) return fail(SF_ENOMEM, "host allocation failed");
    struct Cleanup {
        sf_scene **s;
        ~Cleanup()
        {
            if (*s) release(*s);
        }
    } cleanup{&s};

    s->W = d->width;
    s->H = d->height;
    s->N = d->n_peds;
    s->R = d->radius;
    s->R_obs = d->radius_obs < 0 ? d->radius : d->radius_obs;
    s->k = d->k;
    s->alpha = d->alpha;
    s->k_obs = d->k_obs;
    s->alpha_obs = d->alpha_obs;
    s->w_dest = d->w_dest;
    s->seed = d->seed;
    s->start_step = d->start_step;
    s->periodic = d->periodic != 0;
    s->w_heading = d->w_heading;
    s->bw = bw;
    s->bh = bh;
    if (d->heading && s->N) s->h_heading.assign(d->heading, d->heading + s->N);
    if (d->walk_period && s->N) s->h_walk.assign(d->walk_period, d->walk_period + s->N);
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->own_stream = s->stream;
    SF_HIP(hipGetDevice(&s->device), "hipGetDevice");
    SF_HIP(hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, s->device),
           "CU count");
    s->wpr = (s->W + 63) / 64;

    int max_lds = 0;
    SF_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device),
           "LDS size");
    {
        const LawUnits u = law_units(s->R, s->k, s->alpha);
        s->q_unit = u.q;
        s->int_ok = u.int_ok;
        s->int_rounds = u.rounds;
        if (const char *e = std::getenv("SF_FIELD_INT"))
            if (std::atoi(e) == 0) s->int_ok = false;  // speed only: the same field
    }
    const int elem = s->int_ok ? 4 : 8;
    s->lc = sf::pick_list_cfg(s->R, (size_t)max_lds - 1024, elem);
    if (const char *e = std::getenv("SF_TILE")) {
        // launch-shape override "TWxHLxVECxNW[xCAP]"; the field does not
        // depend on it bit for bit, the speed does
        int a = 0, b = 0, v = 0, w = 0, cap = 2048;
        const int got = std::sscanf(e, "%dx%dx%dx%dx%d", &a, &b, &v, &w, &cap);
        if (got != 4 && got != 5)
            return fail(SF_EINVAL, "SF_TILE=%s is not of the form TWxHLxVECxNW[xCAP]", e);
        if (!sf::list_shape_compiled(a, b, w, v, elem) || cap < 1 || cap > (1 << 16))
            return fail(SF_EINVAL, "SF_TILE=%s is not a compiled shape", e);
        s->lc = sf::make_list_cfg(s->R, a, b, w, cap, elem, v);
        if (s->lc.halo_rows > 64 * w)
            return fail(SF_EINVAL, "SF_TILE=%s does not fit radius %d", e, s->R);
    }
    if (s->lc.lds_bytes == 0 || s->lc.lds_bytes > (size_t)max_lds - 1024 ||
        s->lc.list_cap < 2 * s->lc.max_row)
        return fail(SF_EINVAL, "field of radius %d does not fit %d B of LDS", s->R, max_lds);
    // the kernel also holds a few bytes of static LDS
    SF_HIP(sf::set_field_lds_limit((size_t)max_lds - 1024), "LDS limit");
    {
        // as many persistent workgroups as a compute unit holds at once: more
        // would run as a partial second round
        int per_cu = field_blocks_per_cu(s->lc);
        if (const char *e = std::getenv("SF_FIELD_BLOCKS_PER_CU")) {
            // override of the field kernel's persistent workgroups per CU (speed only)
            const int b = std::atoi(e);
            if (b < 1 || b > 64)
                return fail(SF_EINVAL, "SF_FIELD_BLOCKS_PER_CU=%s outside 1..64", e);
            per_cu = b;
        }
        s->lc.grid = s->ncu * per_cu;
    }

    const size_t n = (size_t)s->W * s->H;
    const size_t N = (size_t)s->N;
    s->fp = sf::field_pitch(s->W);
    const size_t nf = (size_t)s->fp * s->H;
    if ((rc = dalloc(s, &s->S, nf, "S")) || (rc = dalloc(s, &s->P, nf, "P")) ||
        (rc = dalloc(s, &s->D, n, "D")) || (rc = dalloc(s, &s->exitm, n, "exit mask")) ||
        (rc = dalloc(s, &s->tab, (size_t)s->lc.tab_elems, "phi table")) ||
        (s->int_ok && (rc = dalloc(s, &s->tabi, (size_t)s->lc.tab_elems, "phi table"))) ||
        (rc = dalloc(s, &s->occ, (size_t)s->wpr * s->H, "occupancy")) ||
        (rc = dalloc(s, &s->claims, n, "claims")) || (rc = dalloc(s, &s->key, N, "keys")) ||
        (rc = dalloc(s, &s->pos, N, "positions")) || (rc = dalloc(s, &s->target, N, "targets")) ||
        (rc = dalloc(s, &s->ext, N, "id map")) ||
        (rc = dalloc(s, &s->flags, (N + 3) & ~(size_t)3, "flags")) ||
        (rc = dalloc(s, &s->ctr, sf::kCtrWords, "counters")))
        return rc;
    if (s->bw * s->bh > 1) {
        if ((rc = dalloc(s, &s->bodies, (size_t)s->wpr * s->H, "body bitmap"))) return rc;
        if (!s->periodic && (rc = dalloc(s, &s->obits, (size_t)s->wpr * s->H, "obstacle bitmap")))
            return rc;
    }
    if (!s->h_heading.empty() && (rc = dalloc(s, &s->heading, N, "headings"))) return rc;
    if (!s->h_walk.empty() && (rc = dalloc(s, &s->walk, N, "walk periods"))) return rc;

    hipStream_t st = s->stream;
    SF_HIP(sf::launch_clear_claims(s->claims, n, st), "clear claims");
    SF_HIP(sf::launch_fill_i32(s->target, N, 0, st), "clear targets");
    SF_HIP(sf::launch_fill_i32(reinterpret_cast<int32_t *>(s->flags), (N + 3) / 4, 0, st),
           "clear flags");
    {
        const ListCfg &c = s->lc;
        const std::vector<double> t = stamp_table(s->R, s->k, s->alpha, c.ncols, c.nrows,
                                                  c.stride, c.padx, c.pady, (size_t)c.tab_elems);
        if ((rc = upload_table(s->tab, t, st))) return rc;
        if (s->tabi) {
            const std::vector<int32_t> ti = stamp_table_int(t, s->q_unit);
            SF_HIP(hipMemcpyAsync(s->tabi, ti.data(), ti.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, st),
                   "copy stamp");
            SF_HIP(hipStreamSynchronize(st), "stamp sync");
        }
        // own-field values at axial and diagonal neighbours (FP32 numbers)
        const size_t ia = (size_t)(c.padx + 1) * c.stride + c.pady;
        s->phi_axial = (float)t[ia];
        s->phi_diag = (float)t[ia + 1];
    }
    if ((rc = upload_positions(s, d->pos))) return rc;
    if ((rc = build_statics(s, d->obstacle, d->exit))) return rc;
    if ((rc = setup_launches(s))) return rc;
    if ((rc = reset_counters(s, s->start_step, 0))) return rc;
    if ((rc = rebuild_dynamic(s))) return rc;
    SF_HIP(hipStreamSynchronize(st), "create sync");
    *out = s;
    s = nullptr;  // ownership passes to the caller
    return SF_OK;
}

// The scene's view (passed by value to its per-tick kernels) and the field's
// work items.
int setup_launches(sf_scene *s)
{
    SceneView &v = s->view;
    v = SceneView{};
    v.W = s->W;
    v.H = s->H;
    v.fp = s->fp;
    v.wpr = s->wpr;
    v.N = s->N;
    v.R = s->R;
    v.dec_block0 = 0;
    v.com_block0 = 0;
    v.phi_axial = s->phi_axial;
    v.phi_diag = s->phi_diag;
    v.seed = s->seed;
    v.S = s->S;
    v.P = s->P;
    v.occ = s->occ;
    v.claims = s->claims;
    v.key = s->key;
    v.ctr = s->ctr;
    v.pos = s->pos;
    v.target = s->target;
    v.flags = s->flags;
    v.exitm = s->exitm;
    v.ext = s->ext;
    v.periodic = s->periodic ? 1 : 0;
    v.heading = s->heading;
    v.walk = s->walk;
    v.hw_axis = (float)s->w_heading;
    v.hw_diag = (float)(s->w_heading / std::sqrt(2.0));
    v.ba = (s->bw - 1) / 2;
    v.bb = (s->bh - 1) / 2;
    v.bodies = s->bodies;
    v.obits = s->obits;
    sf::set_view_layout(v, s->lc, s->tab, s->tabi, s->q_unit, s->int_rounds);
    s->fl = sf::field_launch_for(s->lc);
    // one strip per item: workgroup b takes strips b, b + grid, ...
    s->strips_per_block = 1;
    // the dense stencil for small windows in dense crowds: its (2R+1)^2 fmas
    // per su beat the gather once the crowd fills ~15% of the su
    s->dense = s->R >= 1 && s->R <= sf::kDenseMaxRadius &&
               (double)s->N >= 0.15 * (double)s->W * (double)s->H;
    if (const char *e = std::getenv("SF_FIELD_DENSE")) {
        // override (speed only: both kernels give the same field bit for bit)
        const int d = std::atoi(e);
        if (d == 0) s->dense = false;
        if (d == 1) s->dense = s->R >= 1 && s->R <= sf::kDenseMaxRadius;
    }
    return SF_OK;
}

int enqueue_tick(sf_scene *s)
{
    hipStream_t st = s->stream;
    sf::LaunchEvents ev;
    int rc;
    if ((rc = timing_events(s, SF_KERNEL_DECIDE, &ev))) return rc;
    if (s->bodies)
        SF_HIP(sf::launch_decide_body(s->view, st, &ev), "decide");
    else
        SF_HIP(sf::launch_decide_one(s->view, st, &ev), "decide");
    if ((rc = timing_events(s, SF_KERNEL_COMMIT, &ev))) return rc;
    if (s->bodies)
        SF_HIP(sf::launch_commit_body(s->view, st, &ev), "commit");
    else
        SF_HIP(sf::launch_commit_one(s->view, st, &ev), "commit");
    if ((rc = timing_events(s, SF_KERNEL_SUPERPOSE, &ev))) return rc;
    if (s->refresh > 1 && s->since_full + 1 < s->refresh) {
        // P = (P + stamps at the su entered) - stamps at the su left this tick
        if (s->sect_K) {
            sf::SectView u = s->sect_view;
            u.src = s->moved_to;
            u.src2 = s->moved_from;
            SF_HIP(sf::launch_field_sect(u, s->ncu * 8, true, s->sect_image, st, &ev), "update");
        } else {
            SF_HIP(sf::launch_field_update(s->fl, s->view_upd, s->strips_per_block, st, &ev),
                   "update");
        }
        ++s->since_full;
    } else {
        SF_HIP(scene_field(s, s->view, st, &ev), "superpose");
        s->since_full = 0;
    }
    return SF_OK;
}

// Switches a scene between the full superposition every tick (refresh <= 1)
// and the incremental update with a full superposition every `refresh` ticks.
int set_field_update(sf_scene *s, int32_t refresh)
{
    if (refresh > 1 && !s->moved_from) {
        const size_t nwords = (size_t)s->wpr * s->H;
        int rc;
        if ((rc = dalloc(s, &s->moved_from, nwords, "moved bitmap")) ||
            (rc = dalloc(s, &s->moved_to, nwords, "moved bitmap")) ||
            (rc = dalloc(s, &s->phi, (size_t)s->fp * s->H, "pedestrian field")))
            return rc;
        SF_HIP(sf::launch_fill_u64(s->moved_from, nwords, 0ull, s->stream), "clear moves");
        SF_HIP(sf::launch_fill_u64(s->moved_to, nwords, 0ull, s->stream), "clear moves");
    }
    s->refresh = refresh > 1 ? refresh : 0;
    SceneView &v = s->view;
    v.moved_from = s->refresh ? s->moved_from : nullptr;
    v.moved_to = s->refresh ? s->moved_to : nullptr;
    // full superpositions keep the exact pedestrian field while updates use it
    v.phi = s->refresh ? s->phi : nullptr;
    if (s->refresh) {
        // the field kernel with the moved bitmaps as sources, updating phi in place
        s->view_upd = v;
        s->view_upd.occ = s->moved_to;
    }
    // the next tick starts a new refresh period from a full field
    s->since_full = s->refresh;
    SF_HIP(hipStreamSynchronize(s->stream), "field update sync");
    return SF_OK;
}

// Sect of a nonzero offset d: floor(angle / 45 degrees), the angle of d from
// +x (east) toward +y (south) in [0, 360), each sector half-open at its far
// edge; two sects per quadrant.
int offset_sect(int dx, int dy)
{
    if (dx > 0 && dy >= 0) return dy < dx ? 0 : 1;
    if (dx <= 0 && dy > 0) return -dx < dy ? 2 : 3;
    if (dx < 0 && dy <= 0) return -dy < -dx ? 4 : 5;
    return dx < -dy ? 6 : 7;  // dx >= 0, dy < 0
}

// Switches the scene's field to the paper's own path with K slots (K = 0:
// back to the exact gather) and recomputes the field.
int set_field_sect(sf_scene *s, int K, bool keep_image)
{
    const size_t n = (size_t)s->W * s->H;
    int rc;
    if (K != 0) {
        if (s->R > sf::kSectMaxRadius)
            return fail(SF_EINVAL, "radius %d is above %d for the sect path", s->R,
                        sf::kSectMaxRadius);
        // fan-out terms: sect by sect, row-major within a sect, strengths
        // fl32(k |d|^alpha) as in the gather's stamp
        std::vector<int2> terms;
        const int R = s->R;
        for (int sc = 0; sc < 8; ++sc) {
            const size_t first = terms.size();
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx) {
                    if ((dx == 0 && dy == 0) || offset_sect(dx, dy) != sc) continue;
                    const double dist = std::sqrt((double)dx * dx + (double)dy * dy);
                    const float ph = (float)(s->k * std::pow(dist, s->alpha));
                    int2 t;
                    t.x = (dx + 128) | ((dy + 128) << 8) | (sc << 16);
                    std::memcpy(&t.y, &ph, sizeof ph);
                    terms.push_back(t);
                }
            if (terms.size() > first) terms.back().x |= 1 << 20;  // last term of the sect
        }
        const int n_real = (int)terms.size();
        if (!s->sect_terms && (rc = dalloc(s, &s->sect_terms, (size_t)std::max(n_real, 1),
                                           "sect terms")))
            return rc;
        if (!s->phi32 && (rc = dalloc(s, &s->phi32, (size_t)s->fp * s->H, "FP32 field")))
            return rc;
        if (keep_image && !s->image && (rc = dalloc(s, &s->image, 8 * n, "sect image")))
            return rc;
        if (n_real)
            SF_HIP(hipMemcpyAsync(s->sect_terms, terms.data(), terms.size() * sizeof(int2),
                                  hipMemcpyHostToDevice, s->stream),
                   "copy sect terms");
        sf::SectView &v = s->sect_view;
        v = sf::SectView{};
        v.W = s->W;
        v.H = s->H;
        v.fp = s->fp;
        v.wpr = s->wpr;
        v.R = R;
        v.periodic = s->periodic ? 1 : 0;
        v.K = K;
        v.m = (n_real + K - 1) / K;  // zero terms pad the list to m*K
        v.n_real = n_real;
        v.terms = s->sect_terms;
        v.src = v.src2 = s->occ;
        v.S = s->S;
        v.P = s->P;
        v.phi32 = s->phi32;
        v.image = keep_image ? s->image : nullptr;
    }
    s->sect_K = K;
    s->sect_image = K != 0 && keep_image;
    // the next tick of an incremental update starts from a full field
    s->since_full = s->refresh;
    SF_HIP(scene_field(s, s->view, s->stream), "superpose");
    SF_HIP(hipStreamSynchronize(s->stream), "field path sync");
    return SF_OK;
}

// A field array of the scene (rows of pitch fp, elements of `elem` bytes) to
// dense rows of W elements: on the device by a copy kernel, to the host as
// one contiguous copy of the pitched rows, packed on the host.  (A strided
// runtime copy into pageable host memory read back wrong values under a
// kernel-tracing profiler; these two forms do not depend on it.)
int copy_out_rows(const sf_scene *s, void *dst, const void *src, size_t elem, int on_device)
{
    if (!dst) return SF_OK;
    const size_t W = (size_t)s->W, H = (size_t)s->H, fp = (size_t)s->fp;
    if (on_device) {
        SF_HIP(sf::launch_copy_rows(src, s->fp, dst, s->W, s->H, (int)elem, s->stream),
               "copy rows");
        return SF_OK;
    }
    std::vector<unsigned char> tmp(fp * H * elem);
    SF_HIP(hipMemcpyAsync(tmp.data(), src, tmp.size(), hipMemcpyDeviceToHost, s->stream),
           "copy out");
    SF_HIP(hipStreamSynchronize(s->stream), "copy out sync");
    unsigned char *d = static_cast<unsigned char *>(dst);
    for (size_t y = 0; y < H; ++y) std::memcpy(d + y * W * elem, &tmp[y * fp * elem], W * elem);
    return SF_OK;
}

int copy_out(const sf_scene *s, void *dst, const void *src, size_t bytes, int on_device)
{
    if (!dst) return SF_OK;
    if (on_device) {
        SF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s->stream), "copy out");
    } else {
        SF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s->stream), "copy out");
        SF_HIP(hipStreamSynchronize(s->stream), "copy out sync");
    }
    return SF_OK;
}

// ---- batches ---------------------------------------------------------------------

template <typename T>
int balloc(std::vector<void *> &owned, T **p, size_t n, const char *what)
{
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, (n ? n : 1) * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, what);
    owned.push_back(q);
    *p = static_cast<T *>(q);
    return SF_OK;
}

void free_group(GroupLayout &G)
{
    for (void *p : G.bufs) (void)hipFree(p);
    G = GroupLayout{};
}

void free_layout(BatchLayout &L)
{
    for (GroupLayout &G : L.g) free_group(G);
    for (void *p : L.bufs) (void)hipFree(p);
    L = BatchLayout{};
}

void drop_graphs(sf_batch *b)
{
    for (auto &g : b->graphs) {
        (void)hipGraphExecDestroy(g.second.second);
        (void)hipGraphDestroy(g.second.first);
    }
    b->graphs.clear();
}

constexpr int kDefaultSplitRadius = 8;

// Member indices of each group for tiling `t` (groups and splits filled in).
int split_members(const sf_batch *b, sf_batch_tiling *t,
                  std::vector<int> (&members)[SF_MAX_GROUPS])
{
    if (t->groups < 0 || t->groups > SF_MAX_GROUPS)
        return fail(SF_EINVAL, "groups %d outside 0..%d", t->groups, SF_MAX_GROUPS);
    for (int g = 0; g < SF_MAX_GROUPS - 1; ++g)
        if (t->split_radius[g] < 0 || t->split_radius[g] > SF_MAX_RADIUS)
            return fail(SF_EINVAL, "split_radius[%d] = %d outside 0..%d", g, t->split_radius[g],
                        SF_MAX_RADIUS);
    bool given = false;
    for (int g = 0; g < SF_MAX_GROUPS - 1; ++g) given = given || t->split_radius[g] != 0;
    if (!given) {
        // distinct radii with an estimate of their field work: per su a fixed
        // part (S, P, a strip's bookkeeping) plus the sources of a wave's halo
        std::map<int, double> work;
        for (const sf_scene *s : b->scenes) {
            const double su = (double)s->W * s->H, rho = (double)s->N / su;
            work[s->R] += su * (40.0 + rho * (2.0 * s->R + 16) * (2.0 * s->R + 16) / 4.0);
        }
        std::vector<std::pair<int, double>> r(work.begin(), work.end());  // by radius
        int want = t->groups;
        if (want == 0) want = std::min<int>((int)r.size(), SF_MAX_GROUPS);
        if (want == 2 && t->groups == 2) {
            t->split_radius[0] = kDefaultSplitRadius;
        } else if (want > 1) {
            if ((int)r.size() < want)
                return fail(SF_EINVAL, "%d groups for %d distinct radii", want, (int)r.size());
            // merge the neighbouring pair of smallest joint work until `want` remain
            while ((int)r.size() > want) {
                size_t best = 0;
                for (size_t i = 1; i + 1 < r.size(); ++i)
                    if (r[i].second + r[i + 1].second < r[best].second + r[best + 1].second)
                        best = i;
                r[best].first = r[best + 1].first;
                r[best].second += r[best + 1].second;
                r.erase(r.begin() + (long)best + 1);
            }
            for (int g = 0; g + 1 < want; ++g) t->split_radius[g] = r[(size_t)g].first;
        }
        t->groups = want;
    } else if (t->groups == 0) {
        int n = 1;
        while (n < SF_MAX_GROUPS && t->split_radius[n - 1] != 0) ++n;
        t->groups = n;
    }
    if (t->groups == 0) t->groups = 1;
    for (int g = t->groups - 1; g < SF_MAX_GROUPS - 1; ++g) t->split_radius[g] = 0;
    for (int g = 1; g + 1 < t->groups; ++g)
        if (t->split_radius[g] <= t->split_radius[g - 1])
            return fail(SF_EINVAL, "split radii must increase (%d after %d)", t->split_radius[g],
                        t->split_radius[g - 1]);
    for (auto &m : members) m.clear();
    for (int j = 0; j < (int)b->scenes.size(); ++j) {
        const int R = b->scenes[(size_t)j]->R;
        int g = 0;
        while (g + 1 < t->groups && R > t->split_radius[g]) ++g;
        members[g].push_back(j);
    }
    for (int g = 0; g < t->groups; ++g)
        if (members[g].empty())
            return fail(SF_EINVAL, "the split at radii %d/%d/%d leaves group %d empty",
                        t->split_radius[0], t->split_radius[1], t->split_radius[2], g);
    return SF_OK;
}

// Fill in the defaults of group tiling `t` and check it against the group's
// largest radius R; `lc` receives the launch shape at that radius.
int resolve_group_tiling(const sf_batch *b, int R, int elem, sf_group_tiling *t, ListCfg *lc)
{
    const size_t lds_cap = b->max_lds - 1024;
    if (t->tw == 0 && t->hl == 0 && t->vec == 0 && t->nw == 0) {
        const ListCfg d = sf::pick_list_cfg(R, lds_cap, elem);
        t->tw = d.tw;
        t->hl = d.hl;
        t->vec = d.vec;
        t->nw = d.nw;
        if (t->list_cap == 0) t->list_cap = d.list_cap;
    }
    if (t->vec == 0) t->vec = 2;
    if (!sf::list_shape_compiled(t->tw, t->hl, t->nw, t->vec, elem))
        return fail(SF_EINVAL, "tiling %dx%dx%dx%d is not a compiled shape%s", t->tw, t->hl,
                    t->vec, t->nw, t->vec == 4 ? " (vec 4 needs integer stamps)" : "");
    if (t->list_cap == 0) {
        for (int cap = 4096; cap >= 512; cap /= 2) {
            const ListCfg c = sf::make_list_cfg(R, t->tw, t->hl, t->nw, cap, elem, t->vec);
            if (c.lds_bytes <= lds_cap) {
                t->list_cap = cap;
                break;
            }
        }
    }
    if (t->list_cap < 0 || t->list_cap > (1 << 16))
        return fail(SF_EINVAL, "list_cap %d outside 0..65536", t->list_cap);
    const ListCfg c = sf::make_list_cfg(R, t->tw, t->hl, t->nw, t->list_cap, elem, t->vec);
    if (c.list_cap < 2 * c.max_row || c.halo_rows > 64 * t->nw || c.lds_bytes > lds_cap)
        return fail(SF_EINVAL, "tiling %dx%dx%dx%d with list_cap %d does not fit radius %d",
                    t->tw, t->hl, t->vec, t->nw, t->list_cap, R);
    int bpc_max = std::max(1, std::min((int)((160 * 1024) / c.lds_bytes), 32 / t->nw));
    const int resident =
        sf::field_resident_blocks(t->tw, t->hl, t->nw, c.lds_bytes, true, elem, t->vec);
    if (resident > 0) bpc_max = std::min(bpc_max, resident);  // no partial second round
    if (t->blocks_per_cu == 0) t->blocks_per_cu = bpc_max;
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 64)
        return fail(SF_EINVAL, "blocks_per_cu %d outside 1..64", t->blocks_per_cu);
    if (t->items_per_block == 0) t->items_per_block = 8;
    if (t->items_per_block < 1 || t->items_per_block > 4096)
        return fail(SF_EINVAL, "items_per_block %d outside 1..4096", t->items_per_block);
    *lc = c;
    return SF_OK;
}

// Device layout of one group.  `views` (indexed like sf_batch::scenes)
// receives the members' views.
int build_group(sf_batch *b, const std::vector<int> &members, const sf_group_tiling &req,
                GroupLayout *out, std::vector<SceneView> &views)
{
    GroupLayout G;
    struct Guard {
        GroupLayout *G;
        ~Guard()
        {
            if (G) free_group(*G);
        }
    } guard{&G};
    int R = 0;
    bool int_ok = true;  // one launch: integer sums only if every member's law allows them
    for (int j : members) {
        R = std::max(R, b->scenes[(size_t)j]->R);
        int_ok = int_ok && b->scenes[(size_t)j]->int_ok;
    }
    const int elem = int_ok ? 4 : 8;
    G.t = req;
    G.members = members;
    ListCfg lmax;
    int rc = resolve_group_tiling(b, R, elem, &G.t, &lmax);
    if (rc) return rc;
    const sf_group_tiling &t = G.t;
    G.fl = sf::field_launch_for(lmax);
    G.fl.grid = b->ncu * t.blocks_per_cu;
    hipStream_t st = b->stream;

    const int n = (int)members.size();
    std::vector<SceneView> gv((size_t)n);
    std::vector<double> strip_cost((size_t)n);
    std::map<std::tuple<int, double, double>, void *> tables;
    int64_t dec_total = 0, com_total = 0;
    for (int q = 0; q < n; ++q) {
        const sf_scene *s = b->scenes[(size_t)members[(size_t)q]];
        const ListCfg lc = sf::make_list_cfg(s->R, t.tw, t.hl, t.nw, t.list_cap, elem, t.vec);
        const auto key = std::make_tuple(s->R, s->k, s->alpha);
        void *&tab = tables[key];
        if (!tab) {
            const std::vector<double> td = stamp_table(s->R, s->k, s->alpha, lc.ncols, lc.nrows,
                                                       lc.stride, lc.padx, lc.pady,
                                                       (size_t)lc.tab_elems);
            if (elem == 4) {
                int32_t *ti = nullptr;
                if ((rc = balloc(G.bufs, &ti, (size_t)lc.tab_elems, "batch phi table")))
                    return rc;
                const std::vector<int32_t> h = stamp_table_int(td, s->q_unit);
                SF_HIP(hipMemcpyAsync(ti, h.data(), h.size() * sizeof(int32_t),
                                      hipMemcpyHostToDevice, st),
                       "copy stamp");
                SF_HIP(hipStreamSynchronize(st), "stamp sync");
                tab = ti;
            } else {
                double *t64 = nullptr;
                if ((rc = balloc(G.bufs, &t64, (size_t)lc.tab_elems, "batch phi table")))
                    return rc;
                if ((rc = upload_table(t64, td, st))) return rc;
                tab = t64;
            }
        }
        SceneView v = s->view;
        if (elem == 4)
            sf::set_view_layout(v, lc, nullptr, static_cast<const int32_t *>(tab), s->q_unit,
                                s->int_rounds);
        else
            sf::set_view_layout(v, lc, static_cast<const double *>(tab), nullptr, 1.0);
        v.dec_block0 = (int32_t)dec_total;
        v.com_block0 = (int32_t)com_total;
        dec_total += sf::decide_blocks(s->N);
        com_total += sf::commit_blocks(s->N);
        if (dec_total >= INT32_MAX / 2 || com_total >= INT32_MAX / 2)
            return fail(SF_EINVAL, "batch too large for one launch");
        gv[(size_t)q] = v;
        views[(size_t)members[(size_t)q]] = v;
        // relative cost of one strip: its su, plus the sources each wave
        // gathers (density times the wave tile's halo window)
        const double rho = (double)s->N / ((double)s->W * s->H);
        strip_cost[(size_t)q] = (double)lc.tw * lc.wt +
                                4.0 * lc.nw * rho * (lc.tw + 2.0 * s->R) * (lc.th + 2.0 * s->R);
    }
    G.dec_blocks = (int)dec_total;
    G.com_blocks = (int)com_total;
    std::vector<int32_t> dec_scene((size_t)dec_total), com_scene((size_t)com_total);
    for (int q = 0; q < n; ++q) {
        const SceneView &v = gv[(size_t)q];
        const int64_t d1 = q + 1 < n ? gv[(size_t)q + 1].dec_block0 : dec_total;
        const int64_t c1 = q + 1 < n ? gv[(size_t)q + 1].com_block0 : com_total;
        std::fill(dec_scene.begin() + v.dec_block0, dec_scene.begin() + d1, q);
        std::fill(com_scene.begin() + v.com_block0, com_scene.begin() + c1, q);
    }

    // field items: runs of strips of about equal estimated cost, scenes that
    // share a table adjacent (largest radius first), so that a workgroup's
    // successive items rarely reload the table
    double total = 0.0;
    for (int q = 0; q < n; ++q) total += strip_cost[(size_t)q] * gv[(size_t)q].n_strips;
    const double per_item = total / std::max(1.0, (double)G.fl.grid * t.items_per_block);
    std::vector<int> order((size_t)n);
    for (int q = 0; q < n; ++q) order[(size_t)q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        const sf_scene *x = b->scenes[(size_t)members[(size_t)a]];
        const sf_scene *y = b->scenes[(size_t)members[(size_t)c]];
        return std::make_tuple(-x->R, x->k, x->alpha, -strip_cost[(size_t)a]) <
               std::make_tuple(-y->R, y->k, y->alpha, -strip_cost[(size_t)c]);
    });
    std::vector<int32_t> items;
    for (int q : order) {
        const int ns = gv[(size_t)q].n_strips;
        const int per = (int)std::max(
            1.0, std::min((double)ns, std::floor(per_item / strip_cost[(size_t)q] + 0.5)));
        for (int a = 0; a < ns; a += per) {
            items.push_back(q);
            items.push_back(a);
            items.push_back(std::min(ns, a + per));
            items.push_back(0);
        }
    }
    G.n_items = (int)(items.size() / 4);

    if ((rc = balloc(G.bufs, &G.d_views, gv.size(), "batch views")) ||
        (rc = balloc(G.bufs, &G.d_dec_scene, dec_scene.size(), "batch decide map")) ||
        (rc = balloc(G.bufs, &G.d_com_scene, com_scene.size(), "batch commit map")) ||
        (rc = balloc(G.bufs, &G.d_items, items.size(), "batch items")) ||
        (rc = balloc(G.bufs, &G.d_queue, 2, "batch work queue")))
        return rc;
    SF_HIP(sf::launch_fill_i32(reinterpret_cast<int32_t *>(G.d_queue), 2, 0, st), "clear queue");
    SF_HIP(hipMemcpyAsync(G.d_views, gv.data(), gv.size() * sizeof(SceneView),
                          hipMemcpyHostToDevice, st),
           "batch views");
    SF_HIP(hipMemcpyAsync(G.d_dec_scene, dec_scene.data(), dec_scene.size() * 4,
                          hipMemcpyHostToDevice, st),
           "batch decide map");
    SF_HIP(hipMemcpyAsync(G.d_com_scene, com_scene.data(), com_scene.size() * 4,
                          hipMemcpyHostToDevice, st),
           "batch commit map");
    SF_HIP(hipMemcpyAsync(G.d_items, items.data(), items.size() * 4, hipMemcpyHostToDevice, st),
           "batch items");
    SF_HIP(hipStreamSynchronize(st), "batch layout sync");
    *out = G;
    guard.G = nullptr;
    return SF_OK;
}

int build_layout(sf_batch *b, const sf_batch_tiling *req, BatchLayout *out)
{
    BatchLayout L;
    struct Guard {
        BatchLayout *L;
        ~Guard()
        {
            if (L) free_layout(*L);
        }
    } guard{&L};
    L.t = req ? *req : sf_batch_tiling{};
    std::vector<int> members[SF_MAX_GROUPS];
    int rc = split_members(b, &L.t, members);
    if (rc) return rc;
    L.n_groups = L.t.groups;
    std::vector<SceneView> views(b->scenes.size());
    for (int gi = 0; gi < L.n_groups; ++gi) {
        if ((rc = build_group(b, members[gi], L.t.group[gi], &L.g[gi], views))) return rc;
        L.t.group[gi] = L.g[gi].t;
    }
    for (int gi = L.n_groups; gi < SF_MAX_GROUPS; ++gi) L.t.group[gi] = sf_group_tiling{};
    if ((rc = balloc(L.bufs, &L.d_all, views.size(), "batch views")) ||
        (rc = balloc(L.bufs, &L.d_totals, views.size() * 16, "batch totals")))
        return rc;
    SF_HIP(hipMemcpyAsync(L.d_all, views.data(), views.size() * sizeof(SceneView),
                          hipMemcpyHostToDevice, b->stream),
           "batch views");
    SF_HIP(hipStreamSynchronize(b->stream), "batch layout sync");
    *out = L;
    guard.L = nullptr;
    return SF_OK;
}

int group_field(const GroupLayout &G, hipStream_t st, const sf::LaunchEvents *ev = nullptr)
{
    SF_HIP(sf::launch_field(G.fl, G.d_views, G.d_items, G.n_items, G.d_queue, st, ev),
           "batch field");
    return SF_OK;
}

int group_tick(const GroupLayout &G, hipStream_t st)
{
    SF_HIP(sf::launch_decide_claim(G.d_views, G.d_dec_scene, G.dec_blocks, st),
           "batch decide");
    SF_HIP(sf::launch_commit(G.d_views, G.d_com_scene, G.com_blocks, st), "batch commit");
    return group_field(G, st);
}

// `k` ticks of every group: group 0 on `main`, group g > 0 on aux[g - 1],
// forked from and joined back into `main` (the groups share no scene).
int batch_ticks(const sf_batch *b, int k, hipStream_t main, const hipStream_t *aux)
{
    const BatchLayout &L = b->cur;
    int rc;
    if (L.n_groups > 1) {
        SF_HIP(hipEventRecord(b->fork, main), "fork");
        for (int g = 1; g < L.n_groups; ++g)
            SF_HIP(hipStreamWaitEvent(aux[g - 1], b->fork, 0), "fork wait");
    }
    for (int g = 0; g < L.n_groups; ++g) {
        hipStream_t st = g == 0 ? main : aux[g - 1];
        for (int i = 0; i < k; ++i)
            if ((rc = group_tick(L.g[g], st))) return rc;
    }
    for (int g = 1; g < L.n_groups; ++g) {
        SF_HIP(hipEventRecord(b->join[g - 1], aux[g - 1]), "join");
        SF_HIP(hipStreamWaitEvent(main, b->join[g - 1], 0), "join wait");
    }
    return SF_OK;
}

// Executable graph of `k` ticks, captured on first use.
int batch_graph(sf_batch *b, int k, hipGraphExec_t *out)
{
    auto it = b->graphs.find(k);
    if (it != b->graphs.end()) {
        *out = it->second.second;
        return SF_OK;
    }
    SF_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "begin capture");
    const int rc = batch_ticks(b, k, b->capture, b->capture_aux);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->capture, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(ei, "graph instantiate");
    }
    b->graphs[k] = std::make_pair(g, x);
    *out = x;
    return SF_OK;
}

constexpr int kGraphTicks = 8;

void destroy_batch_streams(sf_batch *b)
{
    for (int g = 0; g < SF_MAX_GROUPS - 1; ++g) {
        if (b->aux[g]) (void)hipStreamDestroy(b->aux[g]);
        if (b->capture_aux[g]) (void)hipStreamDestroy(b->capture_aux[g]);
        if (b->join[g]) (void)hipEventDestroy(b->join[g]);
    }
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->fork) (void)hipEventDestroy(b->fork);
}

int batch_create(sf_scene *const *scenes, int32_t n, const sf_batch_tiling *tiling,
                 void *hip_stream, sf_batch **out)
{
    if (!scenes || n <= 0) return fail(SF_EINVAL, "a batch needs at least one scene");
    int dev = 0;
    SF_HIP(hipGetDevice(&dev), "hipGetDevice");
    for (int32_t i = 0; i < n; ++i) {
        const sf_scene *s = scenes[i];
        if (!s) return fail(SF_EINVAL, "scene %d is NULL", i);
        if (s->batch) return fail(SF_EINVAL, "scene %d already belongs to a batch", i);
        if (s->refresh)
            return fail(SF_EINVAL, "scene %d uses the incremental field update", i);
        if (s->bodies)
            return fail(SF_EINVAL, "scene %d has bodies larger than one su", i);
        if (s->sect_K)
            return fail(SF_EINVAL, "scene %d uses the sect field path", i);
        if (s->device != dev) return fail(SF_EINVAL, "scene %d is on device %d, not %d", i, s->device, dev);
        for (int32_t j = 0; j < i; ++j)
            if (scenes[j] == s) return fail(SF_EINVAL, "scene %d is listed twice", i);
    }
    sf_batch *b = new (std::nothrow) sf_batch;
    if (!b) return fail(SF_ENOMEM, "host allocation failed");
    struct Cleanup {
        sf_batch **b;
        ~Cleanup()
        {
            if (*b) {
                free_layout((*b)->cur);
                destroy_batch_streams(*b);
                delete *b;
            }
        }
    } cleanup{&b};
    b->device = dev;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->scenes.assign(scenes, scenes + n);
    SF_HIP(hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    int max_lds = 0;
    SF_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
           "LDS size");
    b->max_lds = (size_t)max_lds;
    SF_HIP(sf::set_field_lds_limit(b->max_lds - 1024), "LDS limit");
    for (int g = 0; g < SF_MAX_GROUPS - 1; ++g) {
        SF_HIP(hipStreamCreateWithFlags(&b->aux[g], hipStreamNonBlocking), "batch stream");
        SF_HIP(hipStreamCreateWithFlags(&b->capture_aux[g], hipStreamNonBlocking),
               "capture stream");
        SF_HIP(hipEventCreateWithFlags(&b->join[g], hipEventDisableTiming), "join event");
    }
    SF_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "capture stream");
    SF_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "fork event");
    for (sf_scene *s : b->scenes) SF_HIP(hipStreamSynchronize(s->stream), "scene sync");
    int rc = build_layout(b, tiling, &b->cur);
    if (rc) return rc;
    for (sf_scene *s : b->scenes) {
        s->batch = b;
        s->stream = b->stream;
    }
    *out = b;
    b = nullptr;
    return SF_OK;
}

// Median of `reps` timed field launches of group layout G.
int time_group_field(sf_batch *b, const GroupLayout &G, int reps, const EventPair &ep,
                     double *med)
{
    std::vector<float> ms((size_t)reps);
    const sf::LaunchEvents lev{ep.a, ep.b};
    for (int r = 0; r < reps; ++r) {
        int rc = group_field(G, b->stream, &lev);
        if (rc) return rc;
        SF_HIP(hipEventSynchronize(ep.b), "tune sync");
        SF_HIP(hipEventElapsedTime(&ms[(size_t)r], ep.a, ep.b), "tune timing");
    }
    std::sort(ms.begin(), ms.end());
    *med = ms[ms.size() / 2];
    return SF_OK;
}

int batch_tune(sf_batch *b, int32_t reps, sf_batch_tiling *chosen)
{
    if (reps < 1 || reps > 1000) return fail(SF_EINVAL, "reps %d outside 1..1000", reps);
    SF_HIP(hipStreamSynchronize(b->stream), "tune sync");
    EventPair ep;
    SF_HIP(hipEventCreateWithFlags(&ep.a, hipEventDisableSystemFence), "hipEventCreate");
    const hipError_t eb = hipEventCreateWithFlags(&ep.b, hipEventDisableSystemFence);
    struct Ev {
        EventPair *p;
        ~Ev()
        {
            if (p->a) (void)hipEventDestroy(p->a);
            if (p->b) (void)hipEventDestroy(p->b);
        }
    } ev_guard{&ep};
    if (eb != hipSuccess) return hip_fail(eb, "hipEventCreate");

    // tw, hl, nw, vec (vec 4 shapes are skipped for groups without integer stamps)
    static const int shapes[][4] = {{16, 2, 4, 2}, {16, 2, 8, 2}, {16, 4, 4, 2}, {16, 4, 8, 2},
                                    {32, 2, 4, 2}, {32, 2, 8, 2}, {32, 4, 4, 2}, {8, 2, 4, 2},
                                    {8, 4, 4, 2},  {16, 4, 4, 4}, {16, 4, 8, 4}, {32, 4, 4, 4},
                                    {8, 4, 4, 4},  {16, 4, 16, 4}, {32, 8, 4, 4}, {16, 8, 4, 4}};
    const int caps[] = {1024, 2048, 4096};
    const int ipbs[] = {2, 8, 32};
    sf_batch_tiling best = b->cur.t;
    std::vector<SceneView> scratch_views(b->scenes.size());
    for (int gi = 0; gi < b->cur.n_groups; ++gi) {
        const std::vector<int> members = b->cur.g[gi].members;
        double best_ms = 1e30;
        for (const auto &sh : shapes) {
            for (int cap : caps) {
                for (int ipb : ipbs) {
                    sf_group_tiling t = b->cur.g[gi].t;
                    t.tw = sh[0];
                    t.hl = sh[1];
                    t.vec = sh[3];
                    t.nw = sh[2];
                    t.list_cap = cap;
                    t.blocks_per_cu = 0;
                    t.items_per_block = ipb;
                    GroupLayout G;
                    if (build_group(b, members, t, &G, scratch_views) != SF_OK)
                        continue;  // shape does not fit this group
                    double med = 0.0;
                    const int rc = time_group_field(b, G, reps, ep, &med);
                    const sf_group_tiling used = G.t;
                    free_group(G);
                    if (rc) return rc;
                    if (med < best_ms) {
                        best_ms = med;
                        best.group[gi] = used;
                    }
                }
            }
        }
    }
    g_last_error.clear();
    BatchLayout L;
    int rc = build_layout(b, &best, &L);
    if (rc) return rc;
    drop_graphs(b);
    free_layout(b->cur);
    b->cur = L;
    if (chosen) *chosen = b->cur.t;
    return SF_OK;
}

// ---- stateless superposition (sf_superpose) -------------------------------------------

// Arguments of a stateless superposition after validation, with its launch
// shape and the scratch it needs: the occupancy bitmap (wpr*H words) and the
// stamp table (lc.tab_elems doubles).
struct SuperposeCall {
    int W = 0, H = 0, R = 0, periodic = 0, n = 0, wpr = 0;
    double k = 1, alpha = -0.5;
    const double *S = nullptr;
    const int32_t *pos = nullptr;
    float *P = nullptr;
    hipStream_t stream = nullptr;
    ListCfg lc;
    size_t lds_limit = 0;
    size_t bitmap_words = 0, tab_bytes = 0;
    double q = 1.0;  // unit of an integer stamp (lc.elem == 4)
    int rounds = 1;  // rounds of 8 integer terms per 32-bit sum
};

int superpose_prepare(int32_t W, int32_t H, int32_t periodic, int32_t R, double k, double alpha,
                      const double *S, const int32_t *pos, int32_t n, float *P, void *hip_stream,
                      SuperposeCall *c)
{
    if (W <= 0 || H <= 0)
        return fail(SF_EINVAL, "grid %d x %d: both sides must be positive", W, H);
    if ((int64_t)W * H >= (int64_t)1 << 31)
        return fail(SF_EINVAL, "grid %d x %d has 2^31 su or more", W, H);
    if (R < 0 || R > SF_MAX_RADIUS) return fail(SF_EINVAL, "radius %d outside 0..%d", R,
                                                SF_MAX_RADIUS);
    if (periodic != 0 && periodic != 1)
        return fail(SF_EINVAL, "periodic = %d is neither 0 nor 1", periodic);
    if (periodic && W < 64) return fail(SF_EINVAL, "periodic grid width %d is below 64", W);
    if (periodic && 2 * R + 1 > std::min(W, H))
        return fail(SF_EINVAL, "periodic grid %d x %d is narrower than the %d-su window", W, H,
                    2 * R + 1);
    if (!std::isfinite(k) || !std::isfinite(alpha))
        return fail(SF_EINVAL, "field parameters must be finite");
    if (n < 0) return fail(SF_EINVAL, "n = %d is negative", n);
    if (n > 0 && !pos) return fail(SF_EINVAL, "pos is NULL with n = %d", n);
    if (!S || !P) return fail(SF_EINVAL, "S and P are required");
    int rc = check_law(R, k, alpha, "pedestrian");
    if (rc) return rc;
    int dev = 0, max_lds = 0;
    SF_HIP(hipGetDevice(&dev), "hipGetDevice");
    SF_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
           "LDS size");
    const LawUnits u = law_units(R, k, alpha);
    c->q = u.q;
    c->rounds = u.rounds;
    c->lc = sf::pick_list_cfg(R, (size_t)max_lds - 1024, u.int_ok ? 4 : 8);
    if (c->lc.lds_bytes == 0 || c->lc.lds_bytes > (size_t)max_lds - 1024 ||
        c->lc.list_cap < 2 * c->lc.max_row)
        return fail(SF_EINVAL, "field of radius %d does not fit %d B of LDS", R, max_lds);
    int ncu = 0;
    SF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    c->lc.grid = ncu * field_blocks_per_cu(c->lc);
    c->lds_limit = (size_t)max_lds - 1024;  // the same limit as the scenes' launches
    c->W = W;
    c->H = H;
    c->R = R;
    c->periodic = periodic;
    c->n = n;
    c->k = k;
    c->alpha = alpha;
    c->S = S;
    c->pos = pos;
    c->P = P;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->wpr = (W + 63) / 64;
    c->bitmap_words = (size_t)c->wpr * H;
    c->tab_bytes = (size_t)c->lc.tab_elems * c->lc.elem;
    return SF_OK;
}

// Enqueues the superposition of `c` on its stream with the given scratch:
// clear the bitmap, mark the positions, fill the stamp, gather.
int superpose_enqueue(const SuperposeCall &c, unsigned long long *bits, void *tab)
{
    const int R = c.R;
    float oct[(SF_MAX_RADIUS + 1) * (SF_MAX_RADIUS + 2) / 2];
    for (int i = 0; i <= R; ++i)
        for (int j = 0; j <= i; ++j) {
            // the same strength as the scene's stamp: fl32(k |d|^alpha)
            const double dist = std::sqrt((double)i * i + (double)j * j);
            oct[i * (i + 1) / 2 + j] =
                (i == 0) ? 0.f : (float)(c.k * std::pow(dist, c.alpha));
        }
    SF_HIP(sf::set_field_lds_limit(c.lds_limit), "LDS limit");
    SF_HIP(sf::launch_fill_u64(bits, c.bitmap_words, 0ull, c.stream), "clear bitmap");
    SF_HIP(sf::launch_occ_mark(c.pos, c.n, bits, c.wpr, c.W, c.W * c.H, c.stream), "mark");
    SF_HIP(sf::launch_stamp_fill(tab, c.lc.elem, c.q, c.lc.tab_elems, c.lc.ncols, c.lc.stride,
                                 c.lc.padx, c.lc.pady, R, oct, c.stream),
           "stamp");
    SceneView v{};
    v.W = c.W;
    v.H = c.H;
    v.fp = c.W;  // the caller's S and P are dense rows
    v.wpr = c.wpr;
    v.R = R;
    v.S = c.S;
    v.P = c.P;
    v.occ = bits;
    v.periodic = c.periodic;
    if (c.lc.elem == 4)
        sf::set_view_layout(v, c.lc, nullptr, static_cast<const int32_t *>(tab), c.q, c.rounds);
    else
        sf::set_view_layout(v, c.lc, static_cast<const double *>(tab), nullptr, 1.0);
    SF_HIP(sf::launch_field_one(sf::field_launch_for(c.lc), v, 1, c.stream), "superpose");
    return SF_OK;
}

// ---- the superposition without allocation (sf_superpose_noalloc) -----------------

// Its scratch lives in a static device array instead: the stamp table (any
// radius's table fits, the LDS bounds it to 160 KiB), then the occupancy
// bitmap of grids of up to 2^20 bitmap words (2^26 su when the width is a
// multiple of 64).  Each device holds its own copy until the process ends.
constexpr size_t kScratchTabDoubles = (size_t)1 << 15;  // 256 KiB
constexpr size_t kScratchBitmapWords = (size_t)1 << 20; // 8 MiB
constexpr int kScratchMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned long long
    scratch[kScratchTabDoubles + kScratchBitmapWords];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (the host-side name of the array is not a device address).
int scratch_address(void **out)
{
    int dev = 0;
    SF_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kScratchMaxDevices)
        return fail(SF_EINVAL, "device %d is beyond the %d devices the static scratch serves",
                    dev, kScratchMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SF_OK;
}

}  // namespace

extern "C" {

int sf_create_scene(const sf_scene_desc *desc, void *hip_stream, sf_scene **out)
{
    g_last_error.clear();
    if (!out) return fail(SF_EINVAL, "out is NULL");
    *out = nullptr;
    try {
        return create(desc, hip_stream, out);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(SF_EDEVICE, "unexpected failure in sf_create_scene");
    }
}

int sf_refresh_field(sf_scene *s, int32_t n_times)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    if (n_times < 0) return fail(SF_EINVAL, "n_times %d is negative", n_times);
    if (s->batch) return fail(SF_EINVAL, "the scene belongs to a batch");
    DeviceGuard g(s->device);
    try {
        for (int32_t i = 0; i < n_times; ++i) {
            sf::LaunchEvents ev;
            int rc;
            if ((rc = timing_events(s, SF_KERNEL_SUPERPOSE, &ev))) return rc;
            SF_HIP(scene_field(s, s->view, s->stream, &ev), "superpose");
        }
        if (n_times > 0) s->since_full = 0;
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
    return SF_OK;
}

int sf_step(sf_scene *s, int32_t n_steps)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    if (n_steps < 0) return fail(SF_EINVAL, "n_steps %d is negative", n_steps);
    if (s->batch) return fail(SF_EINVAL, "the scene belongs to a batch: step the batch");
    DeviceGuard g(s->device);
    try {
        for (int32_t i = 0; i < n_steps; ++i) {
            const int rc = enqueue_tick(s);
            if (rc) return rc;
        }
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
    return SF_OK;
}

int sf_field(const sf_scene *s, float *dst, int dst_on_device)
{
    if (!s || !dst) return fail(SF_EINVAL, "scene or dst is NULL");
    DeviceGuard g(s->device);
    try {
        return copy_out_rows(s, dst, s->P, sizeof(float), dst_on_device);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
}

int sf_positions(const sf_scene *s, int32_t *pos, uint8_t *alive, int dst_on_device)
{
    if (!s || !pos) return fail(SF_EINVAL, "scene or pos is NULL");
    DeviceGuard g(s->device);
    int rc;
    try {
        rc = copy_by_caller_id(s, pos, (const int32_t *)s->pos, dst_on_device);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
    if (rc || !alive) return rc;
    if (dst_on_device) return fail(SF_EINVAL, "alive flags are only produced in host memory");
    for (int i = 0; i < s->N; ++i) alive[i] = pos[i] >= 0;
    return SF_OK;
}

int sf_last_moves(const sf_scene *s, int32_t *target, uint8_t *flags, int dst_on_device)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    DeviceGuard g(s->device);
    try {
        int rc = copy_by_caller_id(s, target, (const int32_t *)s->target, dst_on_device);
        if (rc) return rc;
        return copy_by_caller_id(s, flags, (const uint8_t *)s->flags, dst_on_device,
                                 sf::kPublicFlagBits);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
}

int sf_static_field(const sf_scene *s, double *S, int32_t *D, int dst_on_device)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    DeviceGuard g(s->device);
    const size_t n = (size_t)s->W * s->H;
    int rc;
    try {
        rc = copy_out_rows(s, S, s->S, sizeof(double), dst_on_device);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
    if (rc) return rc;
    return copy_out(s, D, s->D, n * sizeof(int32_t), dst_on_device);
}

int sf_set_state(sf_scene *s, const int32_t *pos, int64_t step)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    if (step < 0) return fail(SF_EINVAL, "step %lld is negative", (long long)step);
    if (s->N > 0 && !pos) return fail(SF_EINVAL, "pos is NULL");
    if (s->batch) return fail(SF_EINVAL, "the scene belongs to a batch");
    DeviceGuard g(s->device);
    try {
        const size_t n = (size_t)s->W * s->H;
        std::vector<uint8_t> obst(n), exitm(n);
        std::vector<double> S(n);
        int rc0 = copy_out_rows(s, S.data(), s->S, sizeof(double), 0);
        if (rc0) return rc0;
        SF_HIP(hipMemcpyAsync(exitm.data(), s->exitm, n, hipMemcpyDeviceToHost, s->stream),
               "copy exits");
        SF_HIP(hipStreamSynchronize(s->stream), "set_state sync");
        for (size_t c = 0; c < n; ++c) obst[c] = std::isinf(S[c]) ? 1 : 0;
        int rc = validate_positions(s->W, s->H, obst.data(), exitm.data(), s->N, pos, true,
                                    (s->bw - 1) / 2, (s->bh - 1) / 2, s->periodic);
        if (rc) return rc;
        int64_t gone = 0;
        for (int i = 0; i < s->N; ++i) gone += pos[i] < 0;
        hipStream_t st = s->stream;
        if ((rc = upload_positions(s, pos))) return rc;
        if ((rc = reset_counters(s, step, gone))) return rc;
        SF_HIP(sf::launch_clear_claims(s->claims, n, st), "clear claims");
        SF_HIP(sf::launch_fill_i32(s->target, (size_t)s->N, 0, st), "clear targets");
        SF_HIP(sf::launch_fill_i32(reinterpret_cast<int32_t *>(s->flags), ((size_t)s->N + 3) / 4,
                                   0, st),
               "clear flags");
        if ((rc = rebuild_dynamic(s))) return rc;
        SF_HIP(hipStreamSynchronize(st), "set_state sync");
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
    return SF_OK;
}

int sf_stats(const sf_scene *s, sf_stats_t *out)
{
    if (!s || !out) return fail(SF_EINVAL, "scene or out is NULL");
    DeviceGuard g(s->device);
    std::vector<unsigned long long> h(sf::kCtrWords);
    SF_HIP(hipMemcpyAsync(h.data(), s->ctr, sf::kCtrWords * 8, hipMemcpyDeviceToHost, s->stream),
           "stats copy");
    SF_HIP(hipStreamSynchronize(s->stream), "stats sync");
    out->step = (int64_t)h[0];
    out->live = counter_sum(h.data(), sf::kLive);
    out->evacuated = counter_sum(h.data(), sf::kEvacuated);
    out->ped_steps = counter_sum(h.data(), sf::kPedSteps);
    out->movers = counter_sum(h.data(), sf::kMovers);
    out->moved = counter_sum(h.data(), sf::kMoved);
    out->tied = counter_sum(h.data(), sf::kTied);
    out->max_claimants = counter_max(h.data(), sf::kMaxClaim);
    return SF_OK;
}

int sf_sync(const sf_scene *s)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    DeviceGuard g(s->device);
    SF_HIP(hipStreamSynchronize(s->stream), "sync");
    return SF_OK;
}

int sf_set_field_update(sf_scene *s, int32_t refresh_ticks)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    if (refresh_ticks < 0 || refresh_ticks > (1 << 20))
        return fail(SF_EINVAL, "refresh_ticks %d outside 0..2^20", refresh_ticks);
    if (s->batch) return fail(SF_EINVAL, "the scene belongs to a batch");
    DeviceGuard g(s->device);
    try {
        return set_field_update(s, refresh_ticks);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
}

int sf_set_field_sect(sf_scene *s, int32_t K, int32_t keep_image)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    if (K != 0 && K != 2 && K != 4 && K != 8 && K != 16)
        return fail(SF_EINVAL, "K = %d is not 0, 2, 4, 8 or 16", K);
    if (s->batch) return fail(SF_EINVAL, "the scene belongs to a batch");
    DeviceGuard g(s->device);
    try {
        return set_field_sect(s, K, keep_image != 0);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
}

int sf_sect_image(const sf_scene *s, float *dst, int dst_on_device)
{
    if (!s || !dst) return fail(SF_EINVAL, "scene or dst is NULL");
    if (!s->sect_image) return fail(SF_EINVAL, "the scene keeps no sect image");
    DeviceGuard g(s->device);
    return copy_out(s, dst, s->image, 8 * (size_t)s->W * s->H * sizeof(float), dst_on_device);
}

int sf_set_timing(sf_scene *s, int enable)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    s->timing = enable != 0;
    if (s->timing)
        for (int k = 0; k < SF_KERNEL_COUNT; ++k) s->ev_used[k] = 0;
    return SF_OK;
}

int sf_kernel_time(const sf_scene *s, int kernel, double *total_ms, int64_t *launches)
{
    if (!s || !total_ms || !launches) return fail(SF_EINVAL, "NULL argument");
    if (kernel < 0 || kernel >= SF_KERNEL_COUNT) return fail(SF_EINVAL, "kernel id %d", kernel);
    DeviceGuard g(s->device);
    SF_HIP(hipStreamSynchronize(s->stream), "timing sync");
    double sum = 0.0;
    for (size_t i = 0; i < s->ev_used[kernel]; ++i) {
        float ms = 0.f;
        SF_HIP(hipEventElapsedTime(&ms, s->ev[kernel][i].a, s->ev[kernel][i].b), "elapsed");
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)s->ev_used[kernel];
    return SF_OK;
}

void sf_destroy_scene(sf_scene *s) { release(s); }

int sf_batch_create(sf_scene *const *scenes, int32_t n_scenes, const sf_batch_tiling *tiling,
                    void *hip_stream, sf_batch **out)
{
    g_last_error.clear();
    if (!out) return fail(SF_EINVAL, "out is NULL");
    *out = nullptr;
    try {
        return batch_create(scenes, n_scenes, tiling, hip_stream, out);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(SF_EDEVICE, "unexpected failure in sf_batch_create");
    }
}

int sf_batch_tune(sf_batch *b, int32_t reps, sf_batch_tiling *chosen)
{
    if (!b) return fail(SF_EINVAL, "batch is NULL");
    if (b->broken) return fail(SF_EINVAL, "a member scene of the batch was destroyed");
    DeviceGuard g(b->device);
    try {
        return batch_tune(b, reps, chosen);
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
}

int sf_batch_get_tiling(const sf_batch *b, sf_batch_tiling *out)
{
    if (!b || !out) return fail(SF_EINVAL, "batch or out is NULL");
    *out = b->cur.t;
    return SF_OK;
}

int sf_batch_step(sf_batch *b, int32_t n_steps)
{
    if (!b) return fail(SF_EINVAL, "batch is NULL");
    if (n_steps < 0) return fail(SF_EINVAL, "n_steps %d is negative", n_steps);
    if (b->broken) return fail(SF_EINVAL, "a member scene of the batch was destroyed");
    DeviceGuard g(b->device);
    try {
        if (n_steps == 1) {
            // a single tick is launched directly (a batch whose membership
            // changes every tick would not reuse a captured graph)
            return batch_ticks(b, 1, b->stream, b->aux);
        }
        while (n_steps > 0) {
            const int k = std::min(n_steps, kGraphTicks);
            hipGraphExec_t x = nullptr;
            const int rc = batch_graph(b, k, &x);
            if (rc) return rc;
            SF_HIP(hipGraphLaunch(x, b->stream), "graph launch");
            n_steps -= k;
        }
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
    return SF_OK;
}

int sf_batch_refresh_field(sf_batch *b, int32_t n_times)
{
    if (!b) return fail(SF_EINVAL, "batch is NULL");
    if (n_times < 0) return fail(SF_EINVAL, "n_times %d is negative", n_times);
    if (b->broken) return fail(SF_EINVAL, "a member scene of the batch was destroyed");
    DeviceGuard g(b->device);
    for (int32_t i = 0; i < n_times; ++i)
        for (int gi = 0; gi < b->cur.n_groups; ++gi) {
            const int rc = group_field(b->cur.g[gi], b->stream);
            if (rc) return rc;
        }
    return SF_OK;
}

int sf_batch_stats(const sf_batch *b, sf_stats_t *out)
{
    if (!b || !out) return fail(SF_EINVAL, "batch or out is NULL");
    if (b->broken) return fail(SF_EINVAL, "a member scene of the batch was destroyed");
    DeviceGuard g(b->device);
    try {
        const size_t n = b->scenes.size();
        std::vector<unsigned long long> h(n * 16);
        SF_HIP(sf::launch_sum_counters(b->cur.d_all, (int)n, b->cur.d_totals, b->stream),
               "batch totals");
        SF_HIP(hipMemcpyAsync(h.data(), b->cur.d_totals, h.size() * 8, hipMemcpyDeviceToHost,
                              b->stream),
               "batch totals copy");
        SF_HIP(hipStreamSynchronize(b->stream), "batch totals sync");
        for (size_t j = 0; j < n; ++j) {
            const unsigned long long *w = &h[j * 16];
            out[j].step = (int64_t)w[0];
            out[j].live = (int64_t)w[1 + sf::kLive];
            out[j].evacuated = (int64_t)w[1 + sf::kEvacuated];
            out[j].ped_steps = (int64_t)w[1 + sf::kPedSteps];
            out[j].movers = (int64_t)w[1 + sf::kMovers];
            out[j].moved = (int64_t)w[1 + sf::kMoved];
            out[j].tied = (int64_t)w[1 + sf::kTied];
            out[j].max_claimants = (int64_t)w[1 + sf::kMaxClaim];
        }
    } catch (const std::bad_alloc &) {
        return fail(SF_ENOMEM, "host allocation failed");
    }
    return SF_OK;
}

int sf_batch_sync(const sf_batch *b)
{
    if (!b) return fail(SF_EINVAL, "batch is NULL");
    DeviceGuard g(b->device);
    SF_HIP(hipStreamSynchronize(b->stream), "batch sync");
    return SF_OK;
}

void sf_batch_destroy(sf_batch *b)
{
    if (!b) return;
    DeviceGuard g(b->device);
    (void)hipStreamSynchronize(b->stream);
    for (sf_scene *s : b->scenes) {
        s->batch = nullptr;
        s->stream = s->own_stream;
    }
    for (hipStream_t a : b->aux)
        if (a) (void)hipStreamSynchronize(a);
    drop_graphs(b);
    free_layout(b->cur);
    destroy_batch_streams(b);
    delete b;
}

int sf_superpose(int32_t width, int32_t height, int32_t periodic, int32_t radius, double k,
                 double alpha, const double *S, const int32_t *pos, int32_t n, float *P,
                 void *hip_stream)
{
    g_last_error.clear();
    SuperposeCall c;
    int rc = superpose_prepare(width, height, periodic, radius, k, alpha, S, pos, n, P,
                               hip_stream, &c);
    if (rc) return rc;
    void *bits = nullptr, *tab = nullptr;
    SF_HIP(hipMallocAsync(&bits, c.bitmap_words * 8, c.stream), "bitmap");
    hipError_t e = hipMallocAsync(&tab, c.tab_bytes, c.stream);
    if (e != hipSuccess) {
        (void)hipFreeAsync(bits, c.stream);
        return hip_fail(e, "stamp table");
    }
    rc = superpose_enqueue(c, static_cast<unsigned long long *>(bits), tab);
    // freed in stream order, after the launches that use them
    const hipError_t e1 = hipFreeAsync(tab, c.stream);
    const hipError_t e2 = hipFreeAsync(bits, c.stream);
    if (rc) return rc;
    SF_HIP(e1, "free stamp table");
    SF_HIP(e2, "free bitmap");
    return SF_OK;
}

int sf_superpose_noalloc(int32_t width, int32_t height, int32_t periodic, int32_t radius,
                         double k, double alpha, const double *S, const int32_t *pos, int32_t n,
                         float *P, void *hip_stream)
{
    g_last_error.clear();
    SuperposeCall c;
    int rc = superpose_prepare(width, height, periodic, radius, k, alpha, S, pos, n, P,
                               hip_stream, &c);
    if (rc) return rc;
    if (c.bitmap_words > kScratchBitmapWords)
        return fail(SF_EINVAL, "grid %d x %d needs %zu bitmap words; the static scratch holds %zu",
                    width, height, c.bitmap_words, kScratchBitmapWords);
    if (c.tab_bytes > kScratchTabDoubles * 8)
        return fail(SF_EINVAL, "the stamp of radius %d needs %zu bytes; the static scratch "
                    "holds %zu", radius, c.tab_bytes, kScratchTabDoubles * 8);
    void *base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    void *tab = base;
    unsigned long long *bits = static_cast<unsigned long long *>(base) + kScratchTabDoubles;
    return superpose_enqueue(c, bits, tab);
}

int sf_device_count(void)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        n = 0;
    }
    return n;
}

const char *sf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
