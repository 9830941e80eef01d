// Internal interface between the C-ABI layer (sf_api.hip) and the kernels
// (sf_kernels.hip).  Not installed; not part of the public boundary.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sf {

// Optional start/stop events recorded by the dispatch itself (profiling
// timestamps of the kernel), for per-kernel timing.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Running totals kept on the device.  Word 0 holds the index of the next
// tick.  Every other total has kSlots copies, each on its own 128-byte line;
// block b adds to copy b % kSlots, so that blocks do not serialise on one
// address, and the host sums the copies.
enum CounterId {
    kLive = 0,    // pedestrians still in the scene (live count at reset + deltas)
    kEvacuated,   // left through an exit
    kPedSteps,    // sum of live counts at tick starts
    kMovers,      // registrations
    kMoved,       // election winners
    kTied,        // FP32 near-tie decisions
    kMaxClaim,    // most registrants of one su in one tick (a running maximum)
    kScratch,     // set-up counts (reachability)
    kNumCounters
};
constexpr int kCtrStride = 16;  // 64-bit words per 128-byte line
constexpr int kSlots = 64;
constexpr size_t kCtrWords = (size_t)(1 + kNumCounters * kSlots) * kCtrStride;
__host__ __device__ inline size_t ctr_index(int id, int slot)
{
    return (size_t)(1 + id * kSlots + slot) * kCtrStride;
}

// Geometry of one launch configuration of the superposition kernel.
// Lane l of a wave owns output column col = l / G and rows rg + G*r
// (rg = l % G, r = 0..HL-1) of a TW x TH wave tile, G = 64 / TW, TH = G*HL.
// The stamp is held column-major in LDS, zero padded so that every
// (output su, source su) pair of a tile and its R-halo indexes inside it:
//   entry(dx, dy) at (dx + padx) * stride + (dy + pady),
//   padx = R + TW - 1, pady = R + TH - 1, stride = 2*pady + 1 rounded up to
//   a multiple G*odd so that a wave's 64 reads fall in 64 distinct banks.
struct SupCfg {
    int tw = 0, hl = 0, g = 0, th = 0;
    int radius = 0;
    int padx = 0, pady = 0;
    int ncols = 0, nrows = 0, stride = 0;
    size_t elem = 4;      // bytes per table entry
    size_t lds_bytes = 0; // table bytes staged in LDS
    int grid = 0;         // persistent workgroups
};

SupCfg make_sup_cfg(int radius, int tw, int hl, size_t elem);

// Launch shape of the per-tick field kernel (source-list gather).
// A workgroup of NW waves covers a TW-column strip of NW*TH rows; wave w owns
// rows [w*TH, (w+1)*TH).  Lane l owns column l % TW and, with rg = l / TW and
// G = 64 / TW, the HL rows rg + G*r (r < HL), so its entries of a source's
// stamp column are G apart and each pair is one paired LDS read (vec = 2);
// or (vec = 4: integer stamps, HL = 4 or 8) the rows HL*rg + r, read four at
// a time by 16-byte loads from one of four copies of the stamp, copy c
// shifted by c entries.
// The stamp is held once, column-major: as integers in units of the law's
// q = 2^(e_min - 23) (elem = 4 bytes; the FP32 strengths are integer
// multiples of q) or as doubles (elem = 8, laws whose strengths span too many
// binades for 32-bit sums of 8 of them):
//   entry (dx, dy) at (dx + padx)*stride + dy + pady,
//   padx = R + TW (one zero column beyond the halo), pady = R + TH - 1,
//   stride >= 2R + TH (a read past the band |dy| <= R lands on zero rows of
//   its own or the neighbouring column; one zero column more at the end),
//   chosen so that each pass of a read hits distinct
//   banks (16 lanes and index mod 16 for doubles, 32 lanes and mod 32 for
//   integers; vec = 4: a multiple of 4, 32 lanes and 16-byte unit mod 32).
// The strip's halo sources are listed in LDS in row-major order; the list
// holds `list_cap` entries and longer halos are processed in several passes.
struct ListCfg {
    int tw = 0, hl = 0, nw = 0;
    int g = 0, th = 0, wt = 0;
    int radius = 0;
    int padx = 0, pady = 0, ncols = 0, nrows = 0, stride = 0;
    int elem = 8;        // bytes per stamp entry: 4 (integers) or 8 (doubles)
    int vec = 2;         // stamp entries per LDS load and lane: 2 or 4
    int tab_elems = 0;   // (ncols + 1) * stride rounded up to whole 16-byte vectors
    int lds_tab = 0;     // stamp entries in LDS: tab_elems, or (vec 4) 4*tab_elems + 4
    int list_cap = 0;
    int max_row = 0;     // most sources one halo row can hold
    int halo_rows = 0;   // most halo rows of one strip
    size_t lds_bytes = 0;
    int grid = 0;
};
ListCfg make_list_cfg(int radius, int tw, int hl, int nw, int list_cap, int elem, int vec = 2);
// Picks the launch shape for radius R that fits `max_lds` bytes of LDS.
ListCfg pick_list_cfg(int radius, size_t max_lds, int elem);
bool list_shape_compiled(int tw, int hl, int nw, int vec = 2, int elem = 4);
// Dynamic LDS limit of the field kernels.
hipError_t set_field_lds_limit(size_t bytes);

// Claim record of one su, 16 bytes: the election word (the smallest key of
// the tick's registrants, ~0 when there is none) and the number of
// registrations, which decide adds and the election's winner reads and clears
// in commit.  Held together, a registrant's two atomics and the winner's reads
// and resets touch one cache line instead of two.
struct ClaimRec {
    unsigned long long word;
    unsigned int regs, pad;
};
hipError_t launch_clear_claims(ClaimRec *c, size_t n, hipStream_t st);

// What the per-tick kernels read of one scene.  A launch covers one or more
// scenes; every scene of a launch has its own view.
struct SceneView {
    int32_t W, H, wpr, N;
    // row pitch (elements) of the su-indexed field arrays S, P and phi; su
    // (x, y) is element y * fp + x of them, while positions and every other
    // su array keep pitch W (see field_pitch)
    int32_t fp;
    int32_t R;
    int32_t dec_block0;  // first workgroup of this scene in the decide launch
    int32_t com_block0;  // first workgroup of this scene in the commit launch
    // field gather layout of this scene's radius under the launch's tile shape
    int32_t tiles_x, n_strips, stride;
    int32_t padx, pady, max_row, tab_elems;
    // integer stamps: rounds of 8 sources the gather sums in 32 bits before it
    // moves the sums into FP64 (8 * int_rounds * max|entry| < 2^31)
    int32_t int_rounds;
    float phi_axial, phi_diag;  // own-field values at axial / diagonal neighbours
    unsigned long long seed;
    const double *tab;          // the stamp as doubles (FP32 strengths), or NULL
    const int32_t *tabi;        // the stamp as integers in units of q, or NULL
    double q;                   // the unit of tabi
    const double *S;            // static field w_dest*D + O (FP64, +inf on obstacles)
    float *P;                   // total field fl32(S + Phi)
    // exact pedestrian field Phi (FP64), kept while the incremental update is
    // on (written by full superpositions, updated in place), else NULL
    double *phi;
    unsigned long long *occ, *key, *ctr;
    // claim record per su (the election word and the tick's registration count)
    ClaimRec *claims;
    // per-pedestrian arrays are indexed by an internal id (pedestrians in
    // row-major order of their positions when the state was set); ext maps
    // it to the caller's id, which keys the election
    int32_t *pos, *target;
    uint8_t *flags;
    const uint8_t *exitm;
    const int32_t *ext;
    // periodic boundary (both axes wrap) and per-pedestrian headings (by
    // internal id, NULL: none) with the FP32 heading weights fl32(w_h) and
    // fl32(w_h / sqrt 2) of aligned and 45-degree moves
    int32_t periodic;
    const uint8_t *heading;
    float hw_axis, hw_diag;
    // walk periods by internal id (NULL: none): pedestrian with caller id e
    // and period p acts on tick t iff (t + e) mod p == 0
    const uint8_t *walk;
    // incremental field update (NULL: the field is recomputed every tick):
    // bitmaps of the su the tick's winners left and entered, set by commit,
    // read by the field update, cleared by the next tick's decide
    unsigned long long *moved_from, *moved_to;
    // pedestrian bodies larger than one su: half-widths (0, 0 = one su), the
    // bitmap of the su the bodies cover and the obstacle bitmap (NULL on a
    // torus); occ keeps the centres, the field's sources
    int32_t ba, bb;
    unsigned long long *bodies;
    const unsigned long long *obits;
};

// Row pitch of a scene's field arrays: W rounded up to a multiple of 32, so
// that every row of P starts on a 128-byte boundary and every row of S on a
// 256-byte one.  A strip's rows are then read and written in whole cache
// lines (a tile of 16 or 32 columns starts at a multiple of 16 columns), not
// in pieces that straddle two lines.
inline int field_pitch(int W) { return (W + 31) & ~31; }

// Field layout fields of `v` for shape `c` (built for the scene's radius):
// the gather reads tabi (unit q) when c.elem == 4, else tab.
void set_view_layout(SceneView &v, const ListCfg &c, const double *tab, const int32_t *tabi,
                     double q, int int_rounds = 1);

// Workgroups of a scene in the decide launches and in a batch's commit launch.
int decide_blocks(int N);
int commit_blocks(int N);

// One field launch over `n_items` work items (int4: scene, first strip,
// end strip, unused), taken by the workgroups from a work queue in the order
// they ask (a single scene's launch: the workgroups on each XCD share a
// contiguous run of the items, in proportion to their number, round robin).
// `tab_max` is the largest lds_tab of the launch's scenes and `halo_max`
// the largest halo row count; both size the dynamic LDS.
struct FieldLaunch {
    int tw = 0, hl = 0, nw = 0;
    int elem = 8;  // stamp entry bytes: 4 = integer sums, 8 = FP64 sums
    int vec = 2;   // stamp entries per LDS load and lane (4: 16-byte loads)
    int list_cap = 0, tab_max = 0, halo_max = 0;
    int grid = 0;
    size_t lds_bytes = 0;
};
FieldLaunch field_launch_for(const ListCfg &c);  // tab_max/halo_max of c, grid = c.grid
// Workgroups of the field kernel of this shape that one compute unit holds at
// once with `lds_bytes` of dynamic LDS (registers and LDS; 0 if unknown).
int field_resident_blocks(int tw, int hl, int nw, size_t lds_bytes, bool multi, int elem,
                          int vec = 2);
size_t field_lds_bytes(const FieldLaunch &f);
// `queue`: two zeroed counters of the launch's work queue (items go to
// workgroups in the order they ask; the launch leaves the counters zeroed).
hipError_t launch_field(const FieldLaunch &f, const SceneView *views, const int32_t *items,
                        int n_items, unsigned int *queue, hipStream_t st,
                        const LaunchEvents *ev = nullptr);
// Single-scene forms: the view is passed by value.  Field item i is strips
// [i*per, (i+1)*per), dealt as above (grid = min(f.grid, items)); decide and
// commit launch the scene's own blocks.
hipError_t launch_field_one(const FieldLaunch &f, const SceneView &view, int per,
                            hipStream_t st, const LaunchEvents *ev = nullptr);
// Incremental update of a single scene's field in one launch: view.occ =
// bitmap of the su entered, view.moved_from = bitmap of the su left, view.phi
// the exact pedestrian field; phi = (phi + Phi(entered)) - Phi(left) in place
// and P = fl32(S + phi), the same bits as launch_field_one.
hipError_t launch_field_update(const FieldLaunch &f, const SceneView &view, int per,
                               hipStream_t st, const LaunchEvents *ev = nullptr);
// Single-scene field by the dense small-radius stencil (radius 1..kDenseMaxRadius),
// bit-identical to launch_field_one; `grid` caps the persistent workgroups.
constexpr int kDenseMaxRadius = 4;
hipError_t launch_field_dense(const SceneView &view, int grid, hipStream_t st,
                              const LaunchEvents *ev = nullptr);
hipError_t launch_decide_one(const SceneView &view, hipStream_t st,
                             const LaunchEvents *ev = nullptr);
hipError_t launch_commit_one(const SceneView &view, hipStream_t st,
                             const LaunchEvents *ev = nullptr);
// Bodies larger than one su (view.ba, view.bb > 0; single scenes): body bitmap
// from the positions, and the tick's decide + claim and commit.
hipError_t launch_body_init(const SceneView &view, hipStream_t st);
hipError_t launch_decide_body(const SceneView &view, hipStream_t st,
                              const LaunchEvents *ev = nullptr);
hipError_t launch_commit_body(const SceneView &view, hipStream_t st,
                              const LaunchEvents *ev = nullptr);

// The paper's own field path (8 sects, fan-out terms, Algorithm 3's K FP32
// slots) of one scene.  terms[i] (i < n_real; the padded count is m*K):
// x = (dx + 128) | (dy + 128) << 8 | sect << 16 | (last term of its sect) << 20,
// y = the FP32 strength's bits; sect by sect, row-major within a sect.
struct SectView {
    int32_t W, H, wpr, R, periodic;
    int32_t fp;  // row pitch of S, P and phi32 (the image planes keep pitch W)
    int32_t K, m, n_real;
    const int2 *terms;
    const unsigned long long *src;   // sources (full field) or the su entered (update)
    const unsigned long long *src2;  // the su left (update), else = src
    const double *S;
    float *P;
    float *phi32;  // the FP32 field, written (full) or updated in place
    float *image;  // 8 planes of W*H sect sums, or NULL
};
constexpr int kSectMaxRadius = 48;
hipError_t launch_field_sect(const SectView &v, int grid, bool update, bool image,
                             hipStream_t st, const LaunchEvents *ev = nullptr);

// Launchers: all enqueue on `st` and return the launch status.
hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t st);
hipError_t launch_mask_to_bits(const uint8_t *mask, unsigned long long *bits, int W, int H,
                               int wpr, hipStream_t st);
// Multi-source BFS of the destination field.  `levels` expansions are
// enqueued starting at `level0`; frontier sizes live in cnt[3] on the device.
// Destination-field BFS: D = 0 on exit su, -1 elsewhere; then launch j =
// 0, 1, ... advances bfs_levels_per_launch() levels over the free-su bitmap
// (obstacle bits obits), reading the visited set and frontier from vis[j & 1]
// and fr[j & 1] (both seeded with the exit bits for j = 0) and writing them
// to the other buffers; active[j % bfs_ring()] > 0 iff a frontier remains
// after launch j (active[0] is cleared before launch 0).
hipError_t launch_bfs_seed(const uint8_t *exitm, int32_t *D, int n, hipStream_t st);
int bfs_levels_per_launch();
int bfs_ring();
hipError_t launch_bfs_block(const unsigned long long *obits, unsigned long long *const vis[2],
                            unsigned long long *const fr[2], int32_t *D, int W, int H, int wpr,
                            int j, unsigned int *active, hipStream_t st);
hipError_t launch_count_unreachable(const uint8_t *obst, const int32_t *D, int n,
                                    unsigned long long *ctr, hipStream_t st);
hipError_t launch_superpose_f64(const SupCfg &c, const unsigned long long *bits, int wpr,
                                const double *tab, double *out, int W, int H, hipStream_t st);
hipError_t set_superpose_lds_limit(size_t f64_bytes);
// S (row pitch fp) from D, O and the obstacle mask (row pitch W)
hipError_t launch_static_S(const int32_t *D, const double *O, const uint8_t *obst,
                           double w_dest, double *S, int W, int H, int fp, hipStream_t st);
hipError_t launch_occ_init(const int32_t *pos, int N, unsigned long long *occ, int wpr, int W,
                           unsigned long long *ctr, hipStream_t st);
// Stateless superposition: bitmap bits of the entries 0 <= pos[i] < nsu (the
// bitmap must be cleared first), and the gather's stamp table (n entries of
// the layout of a ListCfg: doubles, elem = 8, or integers in units of q,
// elem = 4) from the law's strengths over one octant of the window,
// oct[i(i+1)/2 + j] for 0 <= j <= i <= R.
hipError_t launch_occ_mark(const int32_t *pos, int n, unsigned long long *occ, int wpr, int W,
                           int nsu, hipStream_t st);
hipError_t launch_stamp_fill(void *tab, int elem, double q, int n, int ncols, int stride,
                             int padx, int pady, int R, const float *oct, hipStream_t st);
// Decide + claim over `n_blocks` workgroups, decide_blocks(N) per scene.
// `block_scene[b]` names the scene of workgroup b (NULL: every workgroup
// belongs to views[0]).
hipError_t launch_decide_claim(const SceneView *views, const int32_t *block_scene, int n_blocks,
                               hipStream_t st, const LaunchEvents *ev = nullptr);
hipError_t launch_commit(const SceneView *views, const int32_t *block_scene, int n_blocks,
                         hipStream_t st, const LaunchEvents *ev = nullptr);
// Dense rows from a pitched field array: dst[y * W + x] = src[y * fp + x]
// (elements of `elem` = 4 or 8 bytes; both pointers on the device).
hipError_t launch_copy_rows(const void *src, int fp, void *dst, int W, int H, int elem,
                            hipStream_t st);
// dst[ext[i]] = src[i] for i < n (internal to caller order).
hipError_t launch_scatter_i32(const int32_t *src, const int32_t *ext, int32_t *dst, int n,
                              hipStream_t st);
// dst[ext[i]] = src[i] & mask for i < n.
hipError_t launch_scatter_u8(const uint8_t *src, const int32_t *ext, uint8_t *dst, int n,
                             uint8_t mask, hipStream_t st);
// the flag bits a caller sees (SF_FLAG_MOVER | SF_FLAG_WON | SF_FLAG_TIED); the
// kernels keep internal bits above them
constexpr uint8_t kPublicFlagBits = 7u;
// out[j*16 + 0] = step of scene j, out[j*16 + 1 + id] = running total id
// (kMaxClaim: the maximum over the slots, every other total: their sum).
hipError_t launch_sum_counters(const SceneView *views, int n_scenes, unsigned long long *out,
                               hipStream_t st);

}  // namespace sf
