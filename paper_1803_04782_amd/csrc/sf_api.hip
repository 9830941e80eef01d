// C-ABI layer of libsf: scene object, validation, device memory, tick loop.
// The declarations and their contracts are in include/sf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sf.h"
#include "sf_internal.h"

using sf::ListCfg;
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
    double k = 1, alpha = -0.5, k_obs = 1, alpha_obs = -0.5, w_dest = 1;
    unsigned long long seed = 0;
    int64_t start_step = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    int ncu = 0;
    // layout
    int wpr = 0;          // 64-bit words per bitmap row
    int chunk = 4;        // bitmap words per wave in the decide kernel
    ListCfg lc;           // pedestrian field launch shape
    float phi_axial = 0.f, phi_diag = 0.f;
    // device state
    float *S = nullptr, *P = nullptr, *tab = nullptr;
    int32_t *D = nullptr;
    uint8_t *exitm = nullptr;
    unsigned long long *occ = nullptr, *claim = nullptr, *key = nullptr;
    int32_t *pos = nullptr, *target = nullptr, *owner = nullptr;
    uint8_t *flags = nullptr;
    unsigned long long *ctr = nullptr;  // see sf::ctr_index
    std::vector<void *> owned;
    // timing
    bool timing = false;
    std::vector<EventPair> ev[SF_KERNEL_COUNT];
    size_t ev_used[SF_KERNEL_COUNT] = {};
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

int validate(const sf_scene_desc *d)
{
    if (!d) return fail(SF_EINVAL, "descriptor is NULL");
    if (d->width <= 0 || d->height <= 0)
        return fail(SF_EINVAL, "grid %d x %d: both sides must be positive", d->width, d->height);
    if ((int64_t)d->width * d->height >= (int64_t)1 << 31)
        return fail(SF_EINVAL, "grid %d x %d has 2^31 su or more", d->width, d->height);
    if (!d->obstacle || !d->exit) return fail(SF_EINVAL, "obstacle and exit masks are required");
    if (d->n_peds < 0) return fail(SF_EINVAL, "n_peds = %d is negative", d->n_peds);
    if (d->n_peds > 0 && !d->pos) return fail(SF_EINVAL, "pos is NULL with n_peds = %d", d->n_peds);
    if (d->radius < 0 || d->radius > SF_MAX_RADIUS)
        return fail(SF_EINVAL, "radius %d outside 0..%d", d->radius, SF_MAX_RADIUS);
    if (d->radius_obs < -1 || d->radius_obs > SF_MAX_RADIUS)
        return fail(SF_EINVAL, "radius_obs %d outside -1..%d", d->radius_obs, SF_MAX_RADIUS);
    const double params[5] = {d->k, d->alpha, d->k_obs, d->alpha_obs, d->w_dest};
    for (double v : params)
        if (!std::isfinite(v)) return fail(SF_EINVAL, "field parameters must be finite");
    if (d->start_step < 0) return fail(SF_EINVAL, "start_step %lld is negative",
                                       (long long)d->start_step);
    const int64_t n = (int64_t)d->width * d->height;
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

// Pedestrian positions must be in range, on free non-exit su and distinct
// (evacuated = -1 allowed when `allow_gone`).
int validate_positions(int W, int H, const uint8_t *obst, const uint8_t *exitm, int N,
                       const int32_t *pos, bool allow_gone)
{
    const int64_t n = (int64_t)W * H;
    std::vector<uint64_t> seen((size_t)(n + 63) / 64, 0);
    for (int i = 0; i < N; ++i) {
        const int32_t p = pos[i];
        if (p == -1 && allow_gone) continue;
        if (p < 0 || p >= n) return fail(SF_EINVAL, "pedestrian %d at su %d is outside the grid", i, p);
        if (obst[p]) return fail(SF_EINVAL, "pedestrian %d stands on obstacle su %d", i, p);
        if (exitm[p]) return fail(SF_EINVAL, "pedestrian %d stands on exit su %d", i, p);
        uint64_t &w = seen[(size_t)p >> 6];
        const uint64_t bit = 1ull << (p & 63);
        if (w & bit) return fail(SF_EINVAL, "pedestrian %d shares su %d with another", i, p);
        w |= bit;
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

// Occupancy, owner map and live count from the current positions, then the
// field of those positions.  Other counters are left as they are.
int rebuild_dynamic(sf_scene *s)
{
    const size_t nwords = (size_t)s->wpr * s->H;
    SF_HIP(sf::launch_fill_u64(s->occ, nwords, 0ull, s->stream), "clear occupancy");
    SF_HIP(sf::launch_fill_i32(s->owner, (size_t)s->W * s->H, -1, s->stream), "clear owners");
    SF_HIP(sf::launch_occ_init(s->pos, s->N, s->occ, s->wpr, s->W, s->owner, s->ctr, s->stream),
           "occupancy");
    SF_HIP(sf::launch_field_list(s->lc, s->occ, s->wpr, s->tab, s->S, s->P, s->W, s->H, s->stream),
           "superpose");
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

int build_statics(sf_scene *s, const uint8_t *h_obst, const uint8_t *h_exit)
{
    const int W = s->W, H = s->H, n = W * H;
    hipStream_t st = s->stream;
    uint8_t *obst = nullptr;
    int32_t *fa = nullptr, *fb = nullptr;
    unsigned int *cnt = nullptr;
    unsigned long long *obits = nullptr;
    double *tab64 = nullptr, *O = nullptr;
    int rc;
    // temporaries are released right after the statics are built
    const size_t first_tmp = s->owned.size();
    if ((rc = dalloc(s, &obst, (size_t)n, "obstacle mask")) ||
        (rc = dalloc(s, &fa, (size_t)n, "BFS frontier")) ||
        (rc = dalloc(s, &fb, (size_t)n, "BFS frontier")) ||
        (rc = dalloc(s, &cnt, 4, "BFS counters")) ||
        (rc = dalloc(s, &obits, (size_t)s->wpr * H, "obstacle bitmap")))
        return rc;
    SF_HIP(hipMemcpyAsync(obst, h_obst, (size_t)n, hipMemcpyHostToDevice, st), "copy obstacles");
    SF_HIP(hipMemcpyAsync(s->exitm, h_exit, (size_t)n, hipMemcpyHostToDevice, st), "copy exits");

    // destination field: BFS over free su from the exit set
    SF_HIP(sf::launch_fill_i32(reinterpret_cast<int32_t *>(cnt), 4, 0, st), "clear BFS counters");
    SF_HIP(sf::launch_bfs_init(obst, s->exitm, s->D, fa, cnt, n, st), "BFS init");
    const int bfs_grid = std::min(1024, std::max(1, s->ncu * 4));
    const int chunk = 64;
    for (int level = 0;; level += chunk) {
        SF_HIP(sf::launch_bfs_levels(obst, s->D, fa, fb, cnt, W, H, level, chunk, bfs_grid, st),
               "BFS expand");
        unsigned int left = 0;
        SF_HIP(hipMemcpyAsync(&left, &cnt[(level + chunk) % 3], sizeof left,
                              hipMemcpyDeviceToHost, st),
               "BFS frontier size");
        SF_HIP(hipStreamSynchronize(st), "BFS sync");
        if (left == 0) break;
        if (level > n) return fail(SF_EDEVICE, "BFS did not terminate");
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

    // obstacle field in FP64, fused with the destination field into S
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
    SF_HIP(sf::launch_phi_table_f64(tab64, oc, s->k_obs, s->alpha_obs, st), "obstacle table");
    SF_HIP(sf::launch_mask_to_bits(obst, obits, W, H, s->wpr, st), "obstacle bitmap");
    SF_HIP(sf::launch_superpose_f64(ocg, obits, s->wpr, tab64, O, W, H, st), "obstacle field");
    SF_HIP(sf::launch_static_S(s->D, O, obst, s->w_dest, s->S, n, st), "static field");
    SF_HIP(hipStreamSynchronize(st), "statics sync");
    for (size_t i = first_tmp; i < s->owned.size(); ++i) (void)hipFree(s->owned[i]);
    s->owned.resize(first_tmp);
    return SF_OK;
}

int create(const sf_scene_desc *d, void *hip_stream, sf_scene **out)
{
    int rc = validate(d);
    if (rc) return rc;
    if ((rc = validate_positions(d->width, d->height, d->obstacle, d->exit, d->n_peds, d->pos,
                                 false)))
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
    s->stream = static_cast<hipStream_t>(hip_stream);
    SF_HIP(hipGetDevice(&s->device), "hipGetDevice");
    SF_HIP(hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, s->device),
           "CU count");
    s->wpr = (s->W + 63) / 64;
    s->chunk = sf::pick_decide_chunk(s->W, s->H, s->N);

    int max_lds = 0;
    SF_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device),
           "LDS size");
    s->lc = sf::pick_list_cfg(s->R, (size_t)max_lds - 1024);
    if (const char *e = std::getenv("SF_TILE")) {
        // launch-shape override "TWxHLxVECxNW"; the field does not depend on it
        // bit for bit, the speed does
        int a = 0, b = 0, v = 0, w = 0, mode = 1;
        const int got = std::sscanf(e, "%dx%dx%dx%dx%d", &a, &b, &v, &w, &mode);
        if (got != 4 && got != 5)
            return fail(SF_EINVAL, "SF_TILE=%s is not of the form TWxHLxVECxNW[xMODE]", e);
        s->lc = sf::make_list_cfg(s->R, a, b, v, w, mode ? 512 : 2048, mode != 0);
        const bool known = sf::list_shape_compiled(a, b, v, w);
        if (!known || s->lc.halo_rows > (mode ? 3 * 64 : 64 * w))
            return fail(SF_EINVAL, "SF_TILE=%s is not a compiled shape for radius %d", e, s->R);
    }
    if (s->lc.lds_bytes == 0 || s->lc.lds_bytes > (size_t)max_lds - 1024 ||
        s->lc.list_cap < 2 * s->lc.max_row)
        return fail(SF_EINVAL, "field of radius %d does not fit %d B of LDS", s->R, max_lds);
    // the kernel also holds a few bytes of static LDS
    SF_HIP(sf::set_field_list_lds_limit((size_t)max_lds - 1024), "LDS limit");
    {
        int per_cu = (int)std::max<size_t>(1, (size_t)(160 * 1024) / s->lc.lds_bytes);
        per_cu = std::min(per_cu, std::max(1, 32 / (s->lc.nw)));
        s->lc.grid = s->ncu * per_cu;
    }

    const size_t n = (size_t)s->W * s->H;
    const size_t N = (size_t)s->N;
    if ((rc = dalloc(s, &s->S, n, "S")) || (rc = dalloc(s, &s->P, n, "P")) ||
        (rc = dalloc(s, &s->D, n, "D")) || (rc = dalloc(s, &s->exitm, n, "exit mask")) ||
        (rc = dalloc(s, &s->tab, (size_t)s->lc.vec * s->lc.copy_elems, "phi table")) ||
        (rc = dalloc(s, &s->occ, (size_t)s->wpr * s->H, "occupancy")) ||
        (rc = dalloc(s, &s->claim, n, "claims")) || (rc = dalloc(s, &s->key, N, "keys")) ||
        (rc = dalloc(s, &s->pos, N, "positions")) || (rc = dalloc(s, &s->target, N, "targets")) ||
        (rc = dalloc(s, &s->owner, n, "owners")) ||
        (rc = dalloc(s, &s->flags, (N + 3) & ~(size_t)3, "flags")) ||
        (rc = dalloc(s, &s->ctr, sf::kCtrWords, "counters")))
        return rc;

    hipStream_t st = s->stream;
    SF_HIP(sf::launch_fill_u64(s->claim, n, ~0ull, st), "clear claims");
    SF_HIP(sf::launch_fill_i32(s->target, N, 0, st), "clear targets");
    SF_HIP(sf::launch_fill_i32(reinterpret_cast<int32_t *>(s->flags), (N + 3) / 4, 0, st),
           "clear flags");
    SF_HIP(sf::launch_phi_copies(s->tab, s->lc, s->k, s->alpha, st), "phi table");
    if (N)
        SF_HIP(hipMemcpyAsync(s->pos, d->pos, N * sizeof(int32_t), hipMemcpyHostToDevice, st),
               "copy positions");
    if ((rc = build_statics(s, d->obstacle, d->exit))) return rc;
    {
        // own-field values at axial and diagonal neighbours, as the kernels see them
        const size_t ia = (size_t)(s->lc.padx + 1) * s->lc.stride + s->lc.pady;
        const size_t id = ia + 1;
        SF_HIP(hipMemcpyAsync(&s->phi_axial, s->tab + ia, sizeof(float), hipMemcpyDeviceToHost, st),
               "phi copy");
        SF_HIP(hipMemcpyAsync(&s->phi_diag, s->tab + id, sizeof(float), hipMemcpyDeviceToHost, st),
               "phi copy");
    }
    if ((rc = reset_counters(s, s->start_step, 0))) return rc;
    if ((rc = rebuild_dynamic(s))) return rc;
    SF_HIP(hipStreamSynchronize(st), "create sync");
    *out = s;
    s = nullptr;  // ownership passes to the caller
    return SF_OK;
}

int enqueue_tick(sf_scene *s)
{
    hipStream_t st = s->stream;
    sf::LaunchEvents ev;
    int rc;
    if ((rc = timing_events(s, SF_KERNEL_DECIDE, &ev))) return rc;
    SF_HIP(sf::launch_decide_claim(s->chunk, s->occ, s->wpr, s->W, s->H, s->owner, s->P,
                                   s->phi_axial, s->phi_diag, s->seed, s->target, s->key, s->flags,
                                   s->claim, s->ctr, st, &ev),
           "decide");
    if ((rc = timing_events(s, SF_KERNEL_COMMIT, &ev))) return rc;
    SF_HIP(sf::launch_commit(s->N, s->W, s->pos, s->target, s->key, s->flags, s->claim, s->occ,
                             s->wpr, s->owner, s->exitm, s->ctr, st, &ev),
           "commit");
    if ((rc = timing_events(s, SF_KERNEL_SUPERPOSE, &ev))) return rc;
    SF_HIP(sf::launch_field_list(s->lc, s->occ, s->wpr, s->tab, s->S, s->P, s->W, s->H, st, &ev),
           "superpose");
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

int sf_step(sf_scene *s, int32_t n_steps)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    if (n_steps < 0) return fail(SF_EINVAL, "n_steps %d is negative", n_steps);
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
    return copy_out(s, dst, s->P, (size_t)s->W * s->H * sizeof(float), dst_on_device);
}

int sf_positions(const sf_scene *s, int32_t *pos, uint8_t *alive, int dst_on_device)
{
    if (!s || !pos) return fail(SF_EINVAL, "scene or pos is NULL");
    DeviceGuard g(s->device);
    int rc = copy_out(s, pos, s->pos, (size_t)s->N * sizeof(int32_t), dst_on_device);
    if (rc || !alive) return rc;
    if (dst_on_device) return fail(SF_EINVAL, "alive flags are only produced in host memory");
    for (int i = 0; i < s->N; ++i) alive[i] = pos[i] >= 0;
    return SF_OK;
}

int sf_last_moves(const sf_scene *s, int32_t *target, uint8_t *flags, int dst_on_device)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    DeviceGuard g(s->device);
    int rc = copy_out(s, target, s->target, (size_t)s->N * sizeof(int32_t), dst_on_device);
    if (rc) return rc;
    return copy_out(s, flags, s->flags, (size_t)s->N, dst_on_device);
}

int sf_static_field(const sf_scene *s, float *S, int32_t *D, int dst_on_device)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    DeviceGuard g(s->device);
    const size_t n = (size_t)s->W * s->H;
    int rc = copy_out(s, S, s->S, n * sizeof(float), dst_on_device);
    if (rc) return rc;
    return copy_out(s, D, s->D, n * sizeof(int32_t), dst_on_device);
}

int sf_set_state(sf_scene *s, const int32_t *pos, int64_t step)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    if (step < 0) return fail(SF_EINVAL, "step %lld is negative", (long long)step);
    if (s->N > 0 && !pos) return fail(SF_EINVAL, "pos is NULL");
    DeviceGuard g(s->device);
    try {
        const size_t n = (size_t)s->W * s->H;
        std::vector<uint8_t> obst(n), exitm(n);
        std::vector<float> S(n);
        SF_HIP(hipMemcpyAsync(S.data(), s->S, n * sizeof(float), hipMemcpyDeviceToHost, s->stream),
               "copy S");
        SF_HIP(hipMemcpyAsync(exitm.data(), s->exitm, n, hipMemcpyDeviceToHost, s->stream),
               "copy exits");
        SF_HIP(hipStreamSynchronize(s->stream), "set_state sync");
        for (size_t c = 0; c < n; ++c) obst[c] = std::isinf(S[c]) ? 1 : 0;
        int rc = validate_positions(s->W, s->H, obst.data(), exitm.data(), s->N, pos, true);
        if (rc) return rc;
        int64_t gone = 0;
        for (int i = 0; i < s->N; ++i) gone += pos[i] < 0;
        hipStream_t st = s->stream;
        if (s->N)
            SF_HIP(hipMemcpyAsync(s->pos, pos, (size_t)s->N * sizeof(int32_t),
                                  hipMemcpyHostToDevice, st),
                   "copy positions");
        if ((rc = reset_counters(s, step, gone))) return rc;
        SF_HIP(sf::launch_fill_u64(s->claim, n, ~0ull, st), "clear claims");
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
    return SF_OK;
}

int sf_sync(const sf_scene *s)
{
    if (!s) return fail(SF_EINVAL, "scene is NULL");
    DeviceGuard g(s->device);
    SF_HIP(hipStreamSynchronize(s->stream), "sync");
    return SF_OK;
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

const char *sf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
