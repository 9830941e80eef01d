// Internal interface between the C-ABI layer (sf_api.hip) and the kernels
// (sf_kernels.hip).  Not installed; not part of the public boundary.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sf {

// Running totals kept on the device (all 64-bit so they can be updated with
// 64-bit atomics).
struct DevCounters {
    unsigned long long step;       // index of the next tick
    unsigned long long live;       // pedestrians still in the scene
    unsigned long long evacuated;  // left through an exit, in total
    unsigned long long ped_steps;  // sum of live counts at tick starts
    unsigned long long movers;     // sum of registrations
    unsigned long long moved;      // sum of election winners
    unsigned long long tied;       // sum of FP32 near-tie decisions
    unsigned long long scratch;    // set-up counters (BFS, validation)
};

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
// Picks the wave-tile shape used for the FP32 pedestrian field at radius R.
void pick_sup_shape(int radius, int *tw, int *hl);

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
                                    unsigned long long *out, hipStream_t st);
hipError_t launch_superpose_f32(const SupCfg &c, const unsigned long long *bits, int wpr,
                                const float *tab, const float *S, float *P, int W, int H,
                                hipStream_t st);
hipError_t launch_superpose_f64(const SupCfg &c, const unsigned long long *bits, int wpr,
                                const double *tab, double *out, int W, int H, hipStream_t st);
hipError_t set_superpose_lds_limits(size_t f32_bytes, size_t f64_bytes);
hipError_t launch_static_S(const int32_t *D, const double *O, const uint8_t *obst,
                           double w_dest, float *S, int n, hipStream_t st);
hipError_t launch_occ_init(const int32_t *pos, int N, unsigned long long *occ, int wpr, int W,
                           int32_t *bin_count, int bins_x, DevCounters *ctr, hipStream_t st);
hipError_t launch_bin_scan(int32_t *bin_count, int32_t *bin_start, int32_t *bin_cursor,
                           int nb, hipStream_t st);
hipError_t launch_bin_scatter(const int32_t *pos, int N, int W, int bins_x,
                              int32_t *bin_cursor, int32_t *sorted, hipStream_t st);
hipError_t launch_decide_claim(const int32_t *sorted, const int32_t *bin_start, int nb, int N,
                               const int32_t *pos, const float *P,
                               const unsigned long long *occ, int wpr, int W, int H,
                               float phi_axial, float phi_diag, unsigned long long seed,
                               int32_t *target, unsigned long long *key, uint8_t *flags,
                               unsigned long long *claim, DevCounters *ctr, hipStream_t st);
hipError_t launch_commit(int N, int W, int bins_x, int32_t *pos, const int32_t *target,
                         const unsigned long long *key, uint8_t *flags,
                         unsigned long long *claim, unsigned long long *occ, int wpr,
                         const uint8_t *exitm, int32_t *bin_count, DevCounters *ctr,
                         hipStream_t st);

}  // namespace sf
