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

// Launch shape of the per-tick FP32 field kernel (source-list gather).
// A workgroup of NW waves covers a TW-column strip of NW*TH rows; wave w owns
// rows [w*TH, (w+1)*TH).  Lane l owns column l % TW and, with rg = l / TW and
// G = 64 / TW, the HL consecutive rows rg*HL .. rg*HL + HL-1, so its slice of
// a source's stamp column is HL contiguous floats read as HL/VEC aligned
// VEC-wide LDS loads (one contiguous access per lane).  The stamp is kept
// in VEC copies, copy c shifted down by c rows, so that a source at row py
// reads copy (py - pady) mod VEC aligned:
//   copy c, entry (dx, dy) at c*ncols*stride + (dx + padx)*stride + dy + pady + c
//   padx = R + TW (one zero column beyond the halo for padding entries),
//   pady = R + TH - 1, stride >= 2*pady + VEC, stride = VEC * odd (banks).
// The strip's halo sources are listed in LDS in row-major order; the list
// holds `list_cap` entries and longer halos are processed in several passes.
struct ListCfg {
    int tw = 0, hl = 0, vec = 0, nw = 0;
    int g = 0, th = 0, wt = 0;
    int radius = 0;
    int padx = 0, pady = 0, ncols = 0, nrows = 0, stride = 0;
    int copy_elems = 0;  // ncols * stride
    int list_cap = 0;
    int max_row = 0;     // most sources one halo row can hold
    int halo_rows = 0;   // most halo rows of one strip (one wave tile in wave mode)
    bool wave_lists = false;  // wave-private lists (k_field_wave) instead of one per strip
    size_t lds_bytes = 0;
    int grid = 0;
};
ListCfg make_list_cfg(int radius, int tw, int hl, int vec, int nw, int list_cap,
                      bool wave_lists);
// Picks the launch shape for radius R that fits `max_lds` bytes of LDS.
ListCfg pick_list_cfg(int radius, size_t max_lds);
hipError_t launch_phi_copies(float *tab, const ListCfg &c, double k, double alpha,
                             hipStream_t st);
hipError_t launch_field_list(const ListCfg &c, const unsigned long long *bits, int wpr,
                             const float *tab, const float *S, float *P, int W, int H,
                             hipStream_t st, const LaunchEvents *ev = nullptr);
hipError_t set_field_list_lds_limit(size_t bytes);
bool list_shape_compiled(int tw, int hl, int vec, int nw);

// Launchers: all enqueue on `st` and return the launch status.
hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t st);
hipError_t launch_mask_to_bits(const uint8_t *mask, unsigned long long *bits, int W, int H,
                               int wpr, hipStream_t st);
hipError_t launch_phi_table_f32(float *tab, const SupCfg &c, double k, double alpha,
                                hipStream_t st);
hipError_t launch_phi_table_f64(double *tab, const SupCfg &c, double k, double alpha,
                                hipStream_t st);
// Multi-source BFS of the destination field.  `levels` expansions are
// enqueued starting at `level0`; frontier sizes live in cnt[3] on the device.
hipError_t launch_bfs_init(const uint8_t *obst, const uint8_t *exitm, int32_t *D,
                           int32_t *frontier, unsigned int *cnt, int n, hipStream_t st);
hipError_t launch_bfs_levels(const uint8_t *obst, int32_t *D, int32_t *fa, int32_t *fb,
                             unsigned int *cnt, int W, int H, int level0, int levels,
                             int grid, hipStream_t st);
hipError_t launch_count_unreachable(const uint8_t *obst, const int32_t *D, int n,
                                    unsigned long long *ctr, hipStream_t st);
hipError_t launch_superpose_f64(const SupCfg &c, const unsigned long long *bits, int wpr,
                                const double *tab, double *out, int W, int H, hipStream_t st);
hipError_t set_superpose_lds_limit(size_t f64_bytes);
hipError_t launch_static_S(const int32_t *D, const double *O, const uint8_t *obst,
                           double w_dest, float *S, int n, hipStream_t st);
hipError_t launch_occ_init(const int32_t *pos, int N, unsigned long long *occ, int wpr, int W,
                           int32_t *owner, unsigned long long *ctr, hipStream_t st);
// Words of the occupancy bitmap handled per wave by the decide kernel.
int pick_decide_chunk(int W, int H, int N);
hipError_t launch_decide_claim(int chunk, const unsigned long long *occ, int wpr, int W, int H,
                               const int32_t *owner, const float *P, float phi_axial,
                               float phi_diag, unsigned long long seed, int32_t *target,
                               unsigned long long *key, uint8_t *flags,
                               unsigned long long *claim, unsigned long long *ctr,
                               hipStream_t st, const LaunchEvents *ev = nullptr);
hipError_t launch_commit(int N, int W, int32_t *pos, int32_t *target,
                         const unsigned long long *key, uint8_t *flags,
                         unsigned long long *claim, unsigned long long *occ, int wpr,
                         int32_t *owner, const uint8_t *exitm, unsigned long long *ctr,
                         hipStream_t st, const LaunchEvents *ev = nullptr);

}  // namespace sf
