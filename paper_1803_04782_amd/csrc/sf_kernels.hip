// HIP kernels (gfx950) of the social-field tick.
//
// One tick (Algorithm 1 of the paper) runs as
//   bin + decide + claim -> commit -> superpose
// and scene creation as
//   phi tables -> BFS destination field -> obstacle field (FP64) -> S ->
//   occupancy -> superpose.
//
// Field superposition (the role of k-4/k-5 and Algorithms 2/3): every su
// gathers the contributions of the live pedestrians within its R-halo.  The
// occupancy bitmap is the bin structure: counts per su are 0 or 1, so the
// counting sort with one-su bins degenerates to a bitmap, and scanning its
// words row by row enumerates a tile's halo pedestrians in global row-major
// order.  Every su therefore sums its contributions in the same order whatever
// the tiling, which makes the FP32 field reproducible bit for bit.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdint>

#include "sf_internal.h"

namespace sf {

namespace {

constexpr int kDirX[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
constexpr int kDirY[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};

// per-pedestrian flag bits of the last tick (SF_FLAG_* of the public header);
// distinct from the running-total ids kMovers, kMoved, kTied
constexpr uint8_t kFlagMover = 1u, kFlagWon = 2u, kFlagTied = 4u;
// internal: a mover that no other pedestrian can contest (no pedestrian on
// the su around its target but itself) wins without registering
constexpr uint8_t kFlagSolo = 8u;
static_assert((kFlagMover | kFlagWon | kFlagTied) == kPublicFlagBits && !(kFlagSolo & kPublicFlagBits),
              "public flag bits");

// ---- small helpers ------------------------------------------------------------

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Sum of `v` over the block, added by one thread to copy (block % kSlots) of
// running total `id` (skipped when 0).  Every thread of the block must call
// it; it synchronises the block.
template <typename Ctr>
__device__ __forceinline__ void block_sum_add(unsigned int v, Ctr ctr, int id)
{
    __shared__ unsigned int part[16];
    // wave sum by butterfly shuffles
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) part[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
        if (s)
            __hip_atomic_fetch_add(&ctr[ctr_index(id, blockIdx.x % kSlots)], s, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Several running totals at once: the block sum of v[k] is added (one thread,
// copy block % kSlots) to total ids[k]; signed values add in two's
// complement.  One LDS exchange for all of them.  Every thread of the block
// must call it; it synchronises the block.
template <int NV, typename Ctr>
__device__ __forceinline__ void block_sums_add(const int (&v)[NV], Ctr ctr, const int (&ids)[NV])
{
    __shared__ int part[NV][16];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        int x = v[k];
        for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
        if (lane_id() == 0) part[k][wv] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        long long sum = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += part[k][w];
        if (sum)
            __hip_atomic_fetch_add(&ctr[ctr_index(ids[k], blockIdx.x % kSlots)],
                                   (unsigned long long)sum, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Maximum of `v` over the block into copy (block % kSlots) of running total
// `id` by one atomic maximum (skipped when 0).  Every thread of the block must
// call it; it synchronises the block.
template <typename Ctr>
__device__ __forceinline__ void block_max_into(unsigned int v, Ctr ctr, int id)
{
    __shared__ unsigned int part[16];
    for (int d = 32; d >= 1; d >>= 1) v = max(v, (unsigned int)__shfl_xor(v, d));
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) part[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = max(m, (unsigned long long)part[w]);
        if (m)
            __hip_atomic_fetch_max(&ctr[ctr_index(id, blockIdx.x % kSlots)], m, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Maximum of `v` over the wave into copy (workgroup % kSlots) of running total
// `id` by one atomic maximum from lane 0 (skipped when 0); no barrier, so it
// may sit in divergent code only if the whole wave reaches it.
template <typename Ctr>
__device__ __forceinline__ void wave_max_into(unsigned int v, Ctr ctr, int id)
{
    for (int d = 32; d >= 1; d >>= 1) v = max(v, (unsigned int)__shfl_xor(v, d));
    if (lane_id() == 0 && v)
        __hip_atomic_fetch_max(&ctr[ctr_index(id, blockIdx.x % kSlots)], (unsigned long long)v,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pointer into LDS (address space 3): 32-bit byte addresses, ds_* instructions.
template <typename T>
using lds_ptr = const __attribute__((address_space(3))) T *;

// Pointer into device global memory (address space 1).  A pointer read from
// memory (a scene view) is generic to the compiler, and generic accesses
// become flat_* instructions, which also occupy the LDS wait counter; held as
// gptr, its accesses are global_* instructions.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T *p)
{
    return (gptr<T>)p;
}

// Hides the arithmetic origin of a per-lane value from the optimiser (an empty
// asm with a VGPR constraint), so that address expressions built on it are not
// refactored into per-source multiplications.
__device__ __forceinline__ int opaque_lane(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11), word 0 of
// the output.  Round: two 32x32->64 products with 0xD2511F53 (word 0) and
// 0xCD9E8D57 (word 2), outputs (hi1 ^ w1 ^ k0, lo1, hi0 ^ w3 ^ k1, lo0); the key
// advances by 0x9E3779B9 / 0xBB67AE85 between rounds.
__device__ __forceinline__ uint32_t philox_w0(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * w0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, w0);
        const uint32_t lo1 = 0xCD9E8D57u * w2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, w2);
        const uint32_t n0 = hi1 ^ w1 ^ k0;
        const uint32_t n2 = hi0 ^ w3 ^ k1;
        w0 = n0;
        w1 = lo1;
        w2 = n2;
        w3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return w0;
}

// ---- fills and masks ----------------------------------------------------------

__global__ void k_fill_u64(unsigned long long *p, size_t n, unsigned long long v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_clear_claims(ClaimRec *c, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        ClaimRec r;
        r.word = ~0ull;
        r.regs = 0u;
        r.pad = 0u;
        c[i] = r;
    }
}

__global__ void k_fill_i32(int32_t *p, size_t n, int32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One thread per 64-bit word of a row-padded bitmap (wpr words per row).
__global__ void k_mask_to_bits(const uint8_t *__restrict__ mask, unsigned long long *__restrict__ bits,
                               int W, int H, int wpr)
{
    const size_t nw = (size_t)wpr * H;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nw;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / wpr), w = (int)(i % wpr);
        const int x0 = w * 64;
        const int n = min(64, W - x0);
        const uint8_t *row = mask + (size_t)y * W + x0;
        unsigned long long b = 0;
        for (int j = 0; j < n; ++j) b |= (unsigned long long)(row[j] != 0) << j;
        bits[i] = b;
    }
}

// ---- destination field: multi-source BFS --------------------------------------

__global__ void k_bfs_seed(const uint8_t *__restrict__ exitm, int32_t *__restrict__ D, int n)
{
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < (size_t)n) D[c] = exitm[c] ? 0 : -1;  // exit su are never obstacles
}

// Level-synchronous BFS on bitmaps (bit x & 63 of word x >> 6 of a row), one
// launch per kBfsLevels levels.  A workgroup owns a tile of kBfsTileWords
// words by kBfsTileRows rows and advances the tile plus a ring one word
// (64 su) wide and kBfsGhost rows high: a level moves every su's error at
// most one su, so after kBfsLevels <= 64 levels the ring absorbed all of it
// and the tile's frontier and visited set are exact.  Per level
//   new = dilate8(frontier) & free & ~visited
// where dilate8 ORs the word with its one-bit shifts (carries from the
// neighbouring words) and then with the rows above and below.  Only the
// frontier is shared (LDS, double-buffered); each thread keeps its three
// words' free and visited bits and the level at which each tile su was
// reached (six bit planes) in registers, and writes D once, after the last
// level.  The visited set and frontier are read from one buffer and the tile's
// words written to the other (workgroups of a launch that run later still
// read the launch's starting state in their ring).  active[j % kBfsRing]
// counts the workgroups whose tile still has a
// frontier after launch j; a launch that finds that count zero for launch
// j - 1 returns at once (the search is over).
constexpr int kBfsTileWords = 4, kBfsTileRows = 256, kBfsGhost = 64, kBfsLevels = 64;
constexpr int kBfsRegW = kBfsTileWords + 2, kBfsRegH = kBfsTileRows + 2 * kBfsGhost;
constexpr int kBfsRowsPer = 3, kBfsThreads = kBfsRegW * kBfsRegH / kBfsRowsPer;  // 768
constexpr int kBfsRing = 4;
static_assert(kBfsGhost >= kBfsLevels && 64 >= kBfsLevels, "ghost ring narrower than a launch");
static_assert(kBfsRegH % kBfsRowsPer == 0, "rows per thread");

__global__ __launch_bounds__(kBfsThreads) void k_bfs_block(
    const unsigned long long *__restrict__ obits, const unsigned long long *__restrict__ vis_in,
    const unsigned long long *__restrict__ fr_in, unsigned long long *__restrict__ vis_out,
    unsigned long long *__restrict__ fr_out, int32_t *__restrict__ D, int W, int H, int wpr, int j,
    unsigned int *active)
{
    __shared__ unsigned long long front[2][kBfsRegH][kBfsRegW];
    const int tid = (int)threadIdx.x;
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) active[(j + 1) % kBfsRing] = 0u;
    if (j > 0 && active[(j + kBfsRing - 1) % kBfsRing] == 0u) return;

    const int c = tid % kBfsRegW, g = tid / kBfsRegW;
    const int wcol = (int)blockIdx.x * kBfsTileWords - 1 + c;
    const int ry0 = (int)blockIdx.y * kBfsTileRows - kBfsGhost;  // region row 0
    const bool col_in = wcol >= 0 && wcol < wpr;
    const bool col_tile = c >= 1 && c <= kBfsTileWords;
    const unsigned long long in_grid =
        (wcol == wpr - 1 && (W & 63)) ? (1ull << (W & 63)) - 1ull : ~0ull;

    unsigned long long fre[kBfsRowsPer], vs[kBfsRowsPer], last[kBfsRowsPer];
    unsigned long long reached[kBfsRowsPer], plane[kBfsRowsPer][6];
#pragma unroll
    for (int i = 0; i < kBfsRowsPer; ++i) {
        const int r = g * kBfsRowsPer + i, y = ry0 + r;
        const bool ok = col_in && y >= 0 && y < H;
        const size_t idx = (size_t)y * wpr + wcol;
        fre[i] = ok ? ~obits[idx] & in_grid : 0ull;
        vs[i] = ok ? vis_in[idx] : 0ull;
        last[i] = ok ? fr_in[idx] : 0ull;
        front[0][r][c] = last[i];
        reached[i] = 0ull;
#pragma unroll
        for (int b = 0; b < 6; ++b) plane[i][b] = 0ull;
    }
    __syncthreads();

    int cur = 0;
    for (int l = 0; l < kBfsLevels; ++l) {
        unsigned long long h[kBfsRowsPer + 2];
#pragma unroll
        for (int k = 0; k < kBfsRowsPer + 2; ++k) {
            const int r = g * kBfsRowsPer - 1 + k;
            unsigned long long v = 0ull;
            if (r >= 0 && r < kBfsRegH) {
                const unsigned long long m = front[cur][r][c];
                const unsigned long long lf = c > 0 ? front[cur][r][c - 1] : 0ull;
                const unsigned long long rt = c < kBfsRegW - 1 ? front[cur][r][c + 1] : 0ull;
                v = m | (m << 1) | (lf >> 63) | (m >> 1) | (rt << 63);
            }
            h[k] = v;
        }
        int any = 0;
#pragma unroll
        for (int i = 0; i < kBfsRowsPer; ++i) {
            const int r = g * kBfsRowsPer + i;
            const unsigned long long nw = (h[i] | h[i + 1] | h[i + 2]) & fre[i] & ~vs[i];
            vs[i] |= nw;
            last[i] = nw;
            front[cur ^ 1][r][c] = nw;
            any |= nw != 0ull;
            reached[i] |= nw;
#pragma unroll
            for (int b = 0; b < 6; ++b) plane[i][b] |= nw & (0ull - (unsigned long long)((l >> b) & 1));
        }
        cur ^= 1;
        if (!__syncthreads_or(any)) break;  // the region's frontier is empty
    }

    // the tile's words: visited set, frontier and D of the su reached here
    int live = 0;
#pragma unroll
    for (int i = 0; i < kBfsRowsPer; ++i) {
        const int r = g * kBfsRowsPer + i, y = ry0 + r;
        if (!col_tile || !col_in || r < kBfsGhost || r >= kBfsGhost + kBfsTileRows || y >= H)
            continue;
        const size_t idx = (size_t)y * wpr + wcol;
        vis_out[idx] = vs[i];
        fr_out[idx] = last[i];
        live |= last[i] != 0ull;
        unsigned long long m = reached[i];
        while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1ull;
            int lv = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) lv |= (int)((plane[i][q] >> b) & 1ull) << q;
            D[(size_t)y * W + wcol * 64 + b] = j * kBfsLevels + lv + 1;
        }
    }
    if (__syncthreads_or(live) && tid == 0) atomicAdd(&active[j % kBfsRing], 1u);
}

__global__ void k_count_unreachable(const uint8_t *__restrict__ obst, const int32_t *__restrict__ D,
                                    int n, unsigned long long *ctr)
{
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool bad = c < (size_t)n && !obst[c] && D[c] < 0;
    block_sum_add(bad ? 1u : 0u, ctr, kScratch);
}

// S = fl64(fl64(w_dest*D) + O), +inf on obstacles: the product is rounded
// before the sum (no fused multiply-add).  D, O and obst have row pitch W, S
// has row pitch fp (its padding columns are left as they are).
__global__ void k_static_S(const int32_t *__restrict__ D, const double *__restrict__ O,
                           const uint8_t *__restrict__ obst, double w_dest, double *__restrict__ S,
                           int W, int H, int fp)
{
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (size_t)W * H) return;
    const size_t y = c / (size_t)W, x = c - y * (size_t)W;
    S[y * (size_t)fp + x] =
        obst[c] ? (double)INFINITY : __dadd_rn(__dmul_rn(w_dest, (double)D[c]), O[c]);
}

// ---- field superposition --------------------------------------------------------

// Persistent kernel: each wave takes TW x TH output tiles.  For every live
// source in the tile's R-halo (bitmap words scanned in row-major order; the
// source coordinates are wave-uniform) each lane adds HL table entries, one
// per owned row, at immediate offsets G*r from a single per-source address.
constexpr int kSupThreads = 256;

// Static fields: out = sum over the set bits of the stamp (FP64 entries holding
// FP32 strengths, so the sums are exact).
template <int TW, int HL>
__global__ __launch_bounds__(kSupThreads) void k_superpose(
    const unsigned long long *__restrict__ bits, int wpr, const double *__restrict__ tab_g,
    int tab_elems, int stride, int padx, int pady, int R, double *__restrict__ out, int W, int H,
    int tiles_x, int n_tiles)
{
    typedef double T;
    constexpr int G = 64 / TW;
    constexpr int TH = G * HL;
    constexpr int NW = kSupThreads / 64;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *tab = reinterpret_cast<T *>(lds_raw);
    for (int i = threadIdx.x; i < tab_elems; i += kSupThreads) tab[i] = tab_g[i];
    __syncthreads();

    const int lane = (int)lane_id();
    // wave index and everything derived from it is wave-uniform: the source
    // scan below runs on the scalar unit
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int col = lane / G, rg = lane % G;
    const int t0 = __builtin_amdgcn_readfirstlane((int)blockIdx.x * NW + wv);
    const int tstep = __builtin_amdgcn_readfirstlane((int)gridDim.x * NW);

    for (int t = t0; t < n_tiles; t += tstep) {
        const int ty = t / tiles_x, tx = t - ty * tiles_x;
        const int x0 = tx * TW, y0 = ty * TH;
        // byte address in LDS of table entry (this lane's su - source at the
        // origin); a source at (px, py) then reads at base - (px*stride + py)*E
        constexpr int E = (int)sizeof(T);
        const int base = opaque_lane((int)(uint32_t)(uintptr_t)((lds_ptr<T>)tab) +
                                     ((x0 + col + padx) * stride + (y0 + rg + pady)) * E);
        T acc[HL];
#pragma unroll
        for (int r = 0; r < HL; ++r) acc[r] = T(0);
        const int ya = max(y0 - R, 0), yb = min(y0 + TH - 1 + R, H - 1);
        const int xa = max(x0 - R, 0), xb = min(x0 + TW - 1 + R, W - 1);
        const int wa = xa >> 6, nwd = (xb >> 6) - wa + 1;  // 1..3 words per halo row
        const unsigned long long ma = ~0ull << (xa & 63);
        const unsigned long long mb = ~0ull >> (63 - (xb & 63));
        // 64 halo rows at a time: lane i holds the masked words of row ya+r0+i
        for (int r0 = ya; r0 <= yb; r0 += 64) {
            const int y = r0 + lane;
            unsigned long long m0 = 0, m1 = 0, m2 = 0;
            if (y <= yb) {
                const unsigned long long *row = bits + (size_t)y * wpr + wa;
                m0 = row[0];
                if (nwd > 1) m1 = row[1];
                if (nwd > 2) m2 = row[2];
            }
            m0 &= ma;
            if (nwd == 1) m0 &= mb;
            if (nwd == 2) m1 &= mb;
            if (nwd == 3) m2 &= mb;
            unsigned long long nz = __ballot((m0 | m1 | m2) != 0ull);
            while (nz) {  // non-empty halo rows, ascending
                const int li = __builtin_ctzll(nz);
                nz &= nz - 1ull;
                const int py = r0 + li;
                const int rbase = base - py * E;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (j >= nwd) break;
                    const unsigned long long mj = j == 0 ? m0 : (j == 1 ? m1 : m2);
                    unsigned long long mw =
                        ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(mj >> 32), li)
                         << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mj, li);
                    const int cbase = ((wa + j) << 6) * stride * E;
                    while (mw) {  // sources of the word, ascending x
                        const int b = __builtin_ctzll(mw);
                        mw &= mw - 1ull;
                        const lds_ptr<T> src = reinterpret_cast<lds_ptr<T>>(
                            (uint32_t)(rbase - (cbase + b * stride * E)));
#pragma unroll
                        for (int r = 0; r < HL; ++r) acc[r] += src[G * r];
                    }
                }
            }
        }
        const int x = x0 + col;
#pragma unroll
        for (int r = 0; r < HL; ++r) {
            const int y = y0 + rg + G * r;
            if (x < W && y < H) out[(size_t)y * W + x] = acc[r];
        }
    }
}

// ---- per-tick field: source-list gather ---------------------------------------------
//
// Exact sums.  A stamp entry is an FP32 number held as a double (the law
// rounded once to FP32), and every contribution is added in FP64.  The
// nonzero strengths of a law span few binades, so every partial sum of a
// window's entries is an exact FP64 number: the pedestrian field Phi at an su
// does not depend on the order or grouping of its terms, and P = fl32(S + Phi)
// with S in FP64 is the same bit for bit whatever the launch shape, batch,
// kernel (gather or dense stencil) or update path that computed it.
//
// A workgroup takes work items (runs of TW-column strips of NW*TH rows, each
// run inside one scene) and for every strip:
//  1. thread t loads the bitmap words of halo row ya + t and counts its sources;
//  2. a block-wide exclusive scan turns the counts into list offsets, so the
//     list holds the strip's halo sources in global row-major order (a
//     counting sort whose bins are halo rows);
//  3. each thread writes its row's entries: an entry is the byte offset that
//     turns a lane's base address into the address of table entry
//     (lane su - source);
//  4. each wave walks the contiguous part of the list that lies within R rows
//     of its own rows: per source one address add, HL/2 paired LDS loads (or
//     HL/4 16-byte loads, VEC = 4) and HL adds per lane.
// Lane l owns column l % TW and, with rg = l / TW and G = 64 / TW, HL rows of
// its wave's TW x TH tile: rows rg + G*r (r < HL), so that its entries of a
// source are G apart in the column-major stamp and two of them make one
// paired load; or (VEC = 4, integer stamps, HL = 4 or 8) rows HL*rg + r, so
// that its entries of a source are adjacent and 16-byte loads read them four
// at a time.  A 16-byte LDS load must be 16-byte aligned, and the start of a
// lane's entries moves with the source's row: the stamp is held four times in
// LDS, copy c shifted by c entries, and a source in row py reads the copy with
// c = (py - pady) mod 4, which puts every lane's entries on a 16-byte boundary
// (lane rows start at multiples of 4 and the stride is a multiple of 4).  The
// copy is folded into the source's list entry.
// A halo with more than list_cap - max_row sources is processed in several
// passes over consecutive row ranges.  The bitmap rows of the next strip
// (possibly of the next item and scene) are requested before the current
// strip is gathered.  The stamp is reloaded into LDS when consecutive items
// belong to scenes with different tables.

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Exclusive prefix sum over the lanes of a wave of counts in [0, 255], and the
// wave total, from eight ballots.
__device__ __forceinline__ int wave_excl_small(int cnt, int &total)
{
    int excl = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const unsigned long long m = __ballot((cnt >> b) & 1);
        const int below = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        excl += below << b;
        tot += __popcll(m) << b;
    }
    total = tot;
    return excl;
}

// smallest r in [0, n] with a[r] >= v (a non-decreasing, a[n] >= v)
__device__ __forceinline__ int lower_bound_lds(const int *a, int n, int v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// The HL stamp entries of one source for this lane (LDS byte address a, rows
// G apart, or with V4 four adjacent integers at a 16-byte aligned address)
// added to acc.
template <int HL, int G, bool V4, typename T>
__device__ __forceinline__ void gather_one(T *acc, uint32_t a)
{
    T v[HL];
    if constexpr (V4) {
        static_assert(HL % 4 == 0 && sizeof(T) == 4, "16-byte loads of four integers");
        typedef const __attribute__((address_space(3))) i32x4 *ptr4;
#pragma unroll
        for (int h = 0; h < HL / 4; ++h) {
            const i32x4 w = *reinterpret_cast<ptr4>(a + 16u * h);
#pragma unroll
            for (int r = 0; r < 4; ++r) v[4 * h + r] = w[r];
        }
    } else {
        typedef const __attribute__((address_space(3))) T *ptr;
        const ptr s = reinterpret_cast<ptr>(a);
#pragma unroll
        for (int r = 0; r < HL; ++r) v[r] = s[G * r];
    }
#pragma unroll
    for (int r = 0; r < HL; ++r) acc[r] += v[r];
}

// The part of a scene's view that the field kernel reads, kept in scalar
// registers (a whole SceneView copy would be placed in private memory).
struct FieldScene {
    int W, H, fp, wpr, R, tiles_x, stride, padx, pady, max_row, tab_vecs, periodic;
    int rounds;  // integer stamps: rounds of 8 sources summed in 32 bits before a flush
    // the stamp (doubles, or integers in units of q), tab_vecs 16-byte vectors
    gptr<const f64x2> tab;
    double q;
    gptr<const double> S;
    gptr<float> P;
    gptr<double> phi;       // exact pedestrian field, kept for the update path (or NULL)
    gptr<const unsigned long long> occ;
    gptr<const unsigned long long> occ2;  // second source bitmap (update launches)
};

template <bool INT>
__device__ __forceinline__ FieldScene field_scene(const SceneView &v)
{
    FieldScene f;
    f.W = v.W;
    f.H = v.H;
    f.fp = v.fp;
    f.wpr = v.wpr;
    f.R = v.R;
    f.tiles_x = v.tiles_x;
    f.stride = v.stride;
    f.padx = v.padx;
    f.pady = v.pady;
    f.max_row = v.max_row;
    f.tab_vecs = INT ? v.tab_elems / 4 : v.tab_elems / 2;
    f.periodic = v.periodic;
    f.rounds = v.int_rounds;
    f.tab = to_global(INT ? reinterpret_cast<const f64x2 *>(v.tabi)
                          : reinterpret_cast<const f64x2 *>(v.tab));
    f.q = v.q;
    f.S = to_global(v.S);
    f.P = to_global(v.P);
    f.phi = to_global(v.phi);
    f.occ = to_global(v.occ);
    f.occ2 = to_global((const unsigned long long *)v.moved_from);
    return f;
}

// `n` (1..64) bits of a bitmap row starting at column s, s + n <= W.
__device__ __forceinline__ unsigned long long row_bits(gptr<const unsigned long long> row, int s,
                                                       int n, int wpr)
{
    const int w = s >> 6, b = s & 63;
    unsigned long long v = row[w] >> b;
    if (b != 0 && w + 1 < wpr) v |= row[w + 1] << (64 - b);
    return n == 64 ? v : v & ((1ull << n) - 1ull);
}

// Word w of a periodic row seen without wrapping: bit j is the su at column
// (64 w + j) mod W (W >= 64, so the 64 columns cross the seam at most once).
__device__ __forceinline__ unsigned long long wrapped_word(gptr<const unsigned long long> row,
                                                           int w, int W, int wpr)
{
    const int x0 = w * 64;
    if (x0 >= 0 && x0 + 64 <= W) return row[w];
    int s = x0 % W;
    s += s < 0 ? W : 0;
    const int n1 = min(64, W - s);
    unsigned long long v = row_bits(row, s, n1, wpr);
    if (n1 < 64) v |= row_bits(row, 0, 64 - n1, wpr) << n1;
    return v;
}

// Work items of a field launch.  MULTI: items[i] from the table and the
// scene views from `views`; otherwise the single scene `one` (a kernel
// argument, no dependent load) and item i = strips [i*per, (i+1)*per).
template <bool MULTI, bool INT>
struct FieldWork {
    const SceneView &one;
    const SceneView *__restrict__ views;
    const int4 *__restrict__ items;
    int per;
    __device__ __forceinline__ int4 item(int i) const
    {
        if constexpr (MULTI) return items[i];
        return make_int4(0, i * per, min(i * per + per, one.n_strips), 0);
    }
    __device__ __forceinline__ FieldScene scene(int j) const
    {
        if constexpr (MULTI) return field_scene<INT>(views[j]);
        return field_scene<INT>(one);
    }
};

// DUAL (single scene only): the incremental update in one launch.  occ = the
// su entered this tick, occ2 = the su left; Phi := (Phi + Phi(occ)) -
// Phi(occ2) in place (exact), P = fl32(S + Phi).  Each bitmap gets its own
// scan, list and gather into its own accumulators.
// INT: the stamp holds each strength as an integer multiple of the law's
// q = 2^(e_min - 23) (4 bytes, half the LDS traffic of a double), summed in
// 32-bit integers that are moved into FP64 accumulators every 8 sources
// (8 * max|strength| / q < 2^31 for such laws, so no partial sum overflows);
// Phi = q * sum, the same exact value, rounded once.  A law whose strengths
// allow it sums several rounds of 8 before moving the sums (the scene's
// int_rounds, with 8 * int_rounds * max|strength| / q < 2^31).  Otherwise the
// stamp holds doubles summed in FP64.
// VEC: stamp entries per LDS load and lane, 2 (paired loads) or 4 (16-byte
// loads; integer stamps, HL a multiple of 4, the stamp held four times).
template <int TW, int HL, int NW, bool MULTI, bool DUAL = false, bool INT = false, int VEC = 2>
__global__ __launch_bounds__(NW * 64) void k_field(SceneView one,
                                                   const SceneView *__restrict__ views,
                                                   const int4 *__restrict__ items, int n_items,
                                                   int per, int tab_max, int list_cap,
                                                   unsigned int *__restrict__ queue)
{
    static_assert(!(DUAL && MULTI), "the update launch covers one scene");
    static_assert(VEC == 2 || (VEC == 4 && INT && HL % 4 == 0),
                  "16-byte loads: integers, HL a multiple of 4");
    constexpr bool V4 = VEC == 4;
    constexpr int NSRC = DUAL ? 2 : 1;
    // sources per round of the gather (rounds of 4 for lanes of 8 rows, which
    // fit 4 waves per SIMD, measured 2-3% slower than rounds of 8 at 3)
    constexpr int RS = 8;
    constexpr int RQ = RS / 4;  // list vectors (4 entries) per round
    using T = std::conditional_t<INT, int, double>;  // a stamp entry
    constexpr uint32_t ES = sizeof(T);
    const FieldWork<MULTI, INT> work{one, views, items, per};
    constexpr int G = 64 / TW, TH = G * HL, WT = NW * TH, NT = NW * 64;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int wave_tot[NW];
    T *tab = reinterpret_cast<T *>(lds_raw);
    int *list = reinterpret_cast<int *>(tab + tab_max);
    int *row_excl = list + list_cap;

    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane % TW, rg = lane / TW;
    // row of this lane's r-th su within its wave's tile
    auto lrow = [&](int r) { return V4 ? HL * rg + r : rg + G * r; };
    const uint32_t tbase = (uint32_t)(uintptr_t)((lds_ptr<T>)tab);

    // Work items of one scene by XCD: workgroup b runs on XCD b mod 8 (each
    // XCD has its own L2).  XCD x owns a contiguous share of the strips, in
    // proportion to its workgroups, and deals it round robin to them, so that
    // neighbouring strips (which share the cache lines of S, P and the bitmap
    // rows) are worked on under one L2.  A batch's items (ordered for load
    // balance) go to workgroups in the order they ask for them, from the
    // counter queue[0]: a batch's groups run concurrently, and a workgroup that
    // starts late behind another group's launch then takes fewer items instead
    // of holding back the end of its own launch.  Every workgroup counts itself
    // out in queue[1] after its last request; the last one resets both
    // counters for the next launch (no other workgroup touches them again).
    __shared__ int next_item;
    auto grab = [&]() -> int {
        if (tid == 0)
            next_item = (int)__hip_atomic_fetch_add(&queue[0], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        // the value is read before the next request: every item spans at
        // least one strip, and a strip has barriers
        __syncthreads();
        return next_item;
    };
    auto finish = [&]() {
        if constexpr (MULTI) {
            if (tid == 0) {
                const unsigned int d = __hip_atomic_fetch_add(&queue[1], 1u, __ATOMIC_ACQ_REL,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                if (d == gridDim.x - 1) {
                    __hip_atomic_store(&queue[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&queue[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    };
    const int NG = (int)gridDim.x, xb = (int)blockIdx.x & 7, kb = (int)blockIdx.x >> 3;
    int gx = NG, item = (int)blockIdx.x, item_end = n_items;
    if constexpr (MULTI) {
        item = grab();
    } else {
        gx = (NG >> 3) + (xb < (NG & 7) ? 1 : 0);           // workgroups on this XCD
        const int sx = xb * (NG >> 3) + min(xb, NG & 7);    // their first logical index
        item_end = (int)((long long)(sx + gx) * n_items / NG);
        item = (int)((long long)sx * n_items / NG) + kb;
    }
    if (item >= item_end) {
        finish();
        return;
    }
    int4 it = work.item(item);
    FieldScene v = work.scene(it.x);
    int t = it.y;
    // this strip's tile column and row (a division per work item, not per strip)
    int ty = t / v.tiles_x, tx = t - ty * v.tiles_x;
    // stamp into LDS, 8 vectors of 16 bytes per thread and batch: each
    // thread's loads are all issued before the stores, so a batch costs one
    // memory round trip.  The loads are unconditional (indices past the end
    // read the last vector again): a load under a branch of its own would get
    // a wait.
    f64x2 *const tab2 = reinterpret_cast<f64x2 *>(tab);
    auto table_load = [&](const FieldScene &s, int i0, f64x2(&r)[8]) {
        const int n2 = s.tab_vecs;
#pragma unroll
        for (int u = 0; u < 8; ++u) r[u] = s.tab[min(i0 + u * NT + tid, n2 - 1)];
    };
    auto table_store = [&](const FieldScene &s, int i0, const f64x2(&r)[8]) {
        const int n2 = s.tab_vecs;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * NT + tid;
            if (i < n2) {
                if constexpr (V4) {
                    // copy c at integer c * (4 * n2 + 1): shifted by c entries
                    const i32x4 w = __builtin_bit_cast(i32x4, r[u]);
                    int *const ti = reinterpret_cast<int *>(tab);
                    reinterpret_cast<i32x4 *>(ti)[i] = w;
#pragma unroll
                    for (int c = 1; c < 4; ++c) {
                        int *const d = ti + c * (4 * n2 + 1) + 4 * i;
                        d[0] = w[0];
                        d[1] = w[1];
                        d[2] = w[2];
                        d[3] = w[3];
                    }
                } else {
                    tab2[i] = r[u];
                }
            }
        }
    };
    auto load_table = [&](const FieldScene &s) {
        for (int i0 = 0; i0 < s.tab_vecs; i0 += 8 * NT) {
            f64x2 r[8];
            table_load(s, i0, r);
            table_store(s, i0, r);
        }
    };

    // Strip geometry: halo rows [ya, ya + nr), halo bitmap words [wa, wa + nwd).
    // On a periodic scene the halo is not clipped: rows and columns outside
    // the grid are those across the opposite edge (coordinates stay unwrapped,
    // so every source's offset from a lane is its nearest image).
    struct Strip {
        int X0, Y0, ya, nr, xa, xb, wa, nwd;
    };
    // strip (tx, ty): strip index ty * tiles_x + tx
    auto strip = [&](const FieldScene &s, int tx, int ty) {
        Strip g;
        g.X0 = tx * TW;
        g.Y0 = ty * WT;
        if (s.periodic) {
            g.ya = g.Y0 - s.R;
            g.nr = min(g.Y0 + WT - 1, s.H - 1) + s.R - g.ya + 1;
            g.xa = g.X0 - s.R;
            g.xb = min(g.X0 + TW - 1, s.W - 1) + s.R;
        } else {
            g.ya = max(g.Y0 - s.R, 0);
            g.nr = min(g.Y0 + WT - 1 + s.R, s.H - 1) - g.ya + 1;
            g.xa = max(g.X0 - s.R, 0);
            g.xb = min(g.X0 + TW - 1 + s.R, s.W - 1);
        }
        g.wa = g.xa >> 6;  // floor, also for the negative columns of a periodic halo
        g.nwd = (g.xb >> 6) - g.wa + 1;
        return g;
    };
    // bitmap words of this thread's halo row of a strip (issued early: the
    // loads stay in flight across the previous strip's work)
    unsigned long long nw_[NSRC][3];
    auto fetch_rows = [&](const FieldScene &s, int tx, int ty) {
#pragma unroll
        for (int src = 0; src < NSRC; ++src) nw_[src][0] = nw_[src][1] = nw_[src][2] = 0;
        const Strip g = strip(s, tx, ty);
        if (tid < g.nr) {
#pragma unroll
            for (int src = 0; src < NSRC; ++src) {
                const gptr<const unsigned long long> bits = src ? s.occ2 : s.occ;
                unsigned long long *n = nw_[src];
                if (s.periodic) {
                    int y = (g.ya + tid) % s.H;
                    y += y < 0 ? s.H : 0;
                    const gptr<const unsigned long long> row = bits + (size_t)y * s.wpr;
                    n[0] = wrapped_word(row, g.wa, s.W, s.wpr);
                    if (g.nwd > 1) n[1] = wrapped_word(row, g.wa + 1, s.W, s.wpr);
                    if (g.nwd > 2) n[2] = wrapped_word(row, g.wa + 2, s.W, s.wpr);
                } else {
                    const gptr<const unsigned long long> row =
                        bits + (size_t)(g.ya + tid) * s.wpr + g.wa;
                    n[0] = row[0];
                    if (g.nwd > 1) n[1] = row[1];
                    if (g.nwd > 2) n[2] = row[2];
                }
            }
        }
    };
    // S (and, for an update, the previous Phi) of this lane's su in a strip:
    // requested one strip ahead, like the halo rows, so that a strip whose
    // gather is short (small radius, sparse crowd) does not wait for them
    double sv_n[HL], pv_n[HL];
    auto fetch_sp = [&](const FieldScene &s, int tx, int ty) {
        const int x = tx * TW + col, y0 = ty * WT + wv * TH;
#pragma unroll
        for (int r = 0; r < HL; ++r) {
            const int y = y0 + lrow(r);
            const size_t c = (size_t)min(y, s.H - 1) * s.fp + min(x, s.W - 1);
            sv_n[r] = s.S[c];
            pv_n[r] = 0.0;
            if constexpr (DUAL) pv_n[r] = s.phi[c];
        }
    };
    {
        // the first batch of the stamp (all of it unless it exceeds 8 vectors
        // per thread), the first strip's halo rows and its S are requested
        // together, in straight-line code, so that their round trips overlap
        f64x2 r[8];
        fetch_rows(v, tx, ty);
        fetch_sp(v, tx, ty);
        table_load(v, 0, r);
        table_store(v, 0, r);
        for (int i0 = 8 * NT; i0 < v.tab_vecs; i0 += 8 * NT) {
            table_load(v, i0, r);
            table_store(v, i0, r);
        }
    }
    __syncthreads();

    for (;;) {
        // the strip after this one: the next of this item, else the first of
        // this workgroup's next item
        int nitem = item, nt = t + 1, ntx = tx + 1, nty = ty;
        if (ntx == v.tiles_x) {
            ntx = 0;
            ++nty;
        }
        int4 nit = it;
        FieldScene nv = v;
        if (nt >= it.z) {
            if constexpr (MULTI)
                nitem = grab();
            else
                nitem = item + gx;
            if (nitem < item_end) {
                nit = work.item(nitem);
                nt = nit.y;
                if (nit.x != it.x) nv = work.scene(nit.x);
                nty = nt / nv.tiles_x;
                ntx = nt - nty * nv.tiles_x;
            }
        }
        const bool more = nitem < item_end;

        const Strip g = strip(v, tx, ty);
        const int W = v.W, H = v.H, R = v.R, stride = v.stride, padx = v.padx, pady = v.pady;
        const int X0 = g.X0, Y0 = g.Y0, y0w = Y0 + wv * TH;
        const int ya = g.ya, nr = g.nr, xa = g.xa, xb = g.xb, wa = g.wa, nwd = g.nwd;
        const int yb = ya + nr - 1;
        const unsigned long long ma = ~0ull << (xa & 63), mb = ~0ull >> (63 - (xb & 63));

        // 1. this thread's halo row (only the first nr threads hold one; whole
        // waves without a row skip the masking)
        const bool wave_rows = wv * 64 < nr;
        unsigned long long mw[NSRC][3];
        int cnts[NSRC];
#pragma unroll
        for (int src = 0; src < NSRC; ++src) {
            unsigned long long m0 = nw_[src][0], m1 = nw_[src][1], m2 = nw_[src][2];
            int cnt = 0;
            if (wave_rows) {
                m0 &= ma;
                if (nwd == 1) m0 &= mb;
                if (nwd == 2) m1 &= mb;
                if (nwd == 3) m2 &= mb;
                cnt = __popcll(m0) + __popcll(m1) + __popcll(m2);
            }
            mw[src][0] = m0;
            mw[src][1] = m1;
            mw[src][2] = m2;
            cnts[src] = cnt;
        }
        // keep the loads below after the use of the prefetched words, so that
        // the wait for those does not also wait for the new requests
        asm volatile("" ::"v"(cnts[0]), "v"(cnts[NSRC - 1]) : "memory");
        // this strip's S (and previous Phi), requested a strip ago; the next
        // strip's halo rows and S are requested now and arrive while this
        // strip is gathered
        const int x = X0 + col;
        double sv[HL], pv[HL];
#pragma unroll
        for (int r = 0; r < HL; ++r) {
            sv[r] = sv_n[r];
            pv[r] = pv_n[r];
        }
        if (more) {
            fetch_rows(nv, ntx, nty);
            fetch_sp(nv, ntx, nty);
        }

        // this wave's halo rows (relative to ya) and per-lane base address
        const int ra = max(y0w - R, ya) - ya;
        const int rb = min(y0w + TH - 1 + R, yb) - ya;
        const uint32_t lb = (uint32_t)opaque_lane(
            (int)(tbase + (uint32_t)((X0 + col + padx) * stride + (y0w + lrow(0) + pady)) * ES));
        // V4: bytes from one stamp copy to the next (each copy is 4 * tab_vecs
        // integers plus one of shift)
        const uint32_t copy_step = (uint32_t)v.tab_vecs * 16u + 4u;
        // accs: the running sums (INT: 32-bit, moved into sums64 by flush())
        T accs[NSRC][HL];
        double sums64[NSRC][HL];
#pragma unroll
        for (int src = 0; src < NSRC; ++src)
#pragma unroll
            for (int r = 0; r < HL; ++r) {
                accs[src][r] = 0;
                sums64[src][r] = 0.0;
            }
        auto flush = [&](int src) {
            if constexpr (INT) {
#pragma unroll
                for (int r = 0; r < HL; ++r) {
                    sums64[src][r] += (double)accs[src][r];
                    accs[src][r] = 0;
                }
            }
        };

#pragma unroll
        for (int src = 0; src < NSRC; ++src) {
            T *acc = accs[src];
            const int cnt = cnts[src];
            const unsigned long long m0 = mw[src][0], m1 = mw[src][1], m2 = mw[src][2];
            // 2. block exclusive scan of the row counts (ballots within a wave);
            // waves that hold no halo row skip the ballots (their counts are 0)
            int wtot = 0, wexcl = 0;
            if (wave_rows) wexcl = wave_excl_small(cnt, wtot);
            if (lane == 0) wave_tot[wv] = wtot;
            __syncthreads();
            int before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int u = wave_tot[w];
                before += w < wv ? u : 0;
                total += u;
            }
            const int excl = before + wexcl;
            if (tid < nr) row_excl[tid] = excl;
            if (tid == 0) row_excl[nr] = total;
            __syncthreads();

            const int cap = list_cap - v.max_row;
            const int npass = total <= cap ? 1 : (total + cap - 1) / cap;
            for (int k = 0; k < npass; ++k) {
                int start = 0, end = total;
                if (npass > 1) {
                    start = row_excl[lower_bound_lds(row_excl, nr, k * cap)];
                    if (k + 1 < npass) end = row_excl[lower_bound_lds(row_excl, nr, (k + 1) * cap)];
                }
                // 3. entries of the rows in this pass: minus the byte offset of
                // the source (px, py) in the column-major stamp, modulo 2^32
                if (tid < nr && cnt > 0 && excl >= start && excl < end) {
                    const uint32_t py = (uint32_t)(ya + tid);
                    // V4: the copy whose shift aligns this row's sources
                    const uint32_t coff =
                        V4 ? (uint32_t)((ya + tid - pady) & 3) * copy_step : 0u;
                    int o = excl - start;
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        unsigned long long mj = j == 0 ? m0 : (j == 1 ? m1 : m2);
                        const int xw = (wa + j) * 64;
                        while (mj) {
                            const int b = __builtin_ctzll(mj);
                            mj &= mj - 1ull;
                            const uint32_t px = (uint32_t)(xw + b);
                            list[o++] = (int)(coff - (px * (uint32_t)stride + py) * ES);
                        }
                    }
                }
                __syncthreads();
                // 4. gather: list entries are read four at a time (one broadcast
                // LDS load), each source costs one address add per lane
                if (ra <= rb) {
                    const int lo = __builtin_amdgcn_readfirstlane(max(row_excl[ra], start) - start);
                    const int hi = __builtin_amdgcn_readfirstlane(min(row_excl[rb + 1], end) - start);
                    int i = lo;
                    for (; i < hi && (i & 3); ++i)
                        gather_one<HL, G, V4>(acc, lb + (uint32_t)list[i]);
                    flush(src);
                    const int4 *list4 = reinterpret_cast<const int4 *>(list);
                    typedef const __attribute__((address_space(3))) T *lds_d;
                    typedef const __attribute__((address_space(3))) i32x4 *lds_4;
                    // the HL entries of a source at LDS byte address ad
                    auto read_at = [&](uint32_t ad, T(&u)[HL]) {
                        if constexpr (V4) {
#pragma unroll
                            for (int h = 0; h < HL / 4; ++h) {
                                const i32x4 w = *reinterpret_cast<lds_4>(ad + 16u * h);
#pragma unroll
                                for (int r = 0; r < 4; ++r) u[4 * h + r] = w[r];
                            }
                        } else {
                            const lds_d sp = reinterpret_cast<lds_d>(ad);
#pragma unroll
                            for (int r = 0; r < HL; ++r) u[r] = sp[G * r];
                        }
                    };
                    // RS sources per round: their table reads are in flight before
                    // the adds, and the next round's entries are read behind them
                    // (reading up to RS entries past the pass stays inside the
                    // allocation: row_excl follows the list).  Integer sums are
                    // moved into FP64 after every 8 * v.rounds sources.
                    if (i + RS <= hi) {
                        int4 e[RQ];
#pragma unroll
                        for (int q = 0; q < RQ; ++q) e[q] = list4[(i >> 2) + q];
                        int pend = 0;  // integer terms per lane since the last flush, / HL
                        for (; i + RS <= hi; i += RS) {
                            // the round's addresses are formed before the next
                            // entries are requested into the same registers
                            uint32_t ad[RS];
#pragma unroll
                            for (int q = 0; q < RQ; ++q) {
                                ad[4 * q] = lb + (uint32_t)e[q].x;
                                ad[4 * q + 1] = lb + (uint32_t)e[q].y;
                                ad[4 * q + 2] = lb + (uint32_t)e[q].z;
                                ad[4 * q + 3] = lb + (uint32_t)e[q].w;
                            }
#pragma unroll
                            for (int u = 0; u < RS; ++u) asm volatile("" : "+v"(ad[u]));
#pragma unroll
                            for (int q = 0; q < RQ; ++q) e[q] = list4[(i >> 2) + RQ + q];
                            // the compiler keeps this order: next entries, table
                            // reads, adds (no wait is implied by the barriers)
                            asm volatile("" ::: "memory");
                            T ur[RS][HL];
#pragma unroll
                            for (int u = 0; u < RS; ++u) read_at(ad[u], ur[u]);
                            asm volatile("" ::: "memory");
#pragma unroll
                            for (int u = 0; u < RS; ++u) {
#pragma unroll
                                for (int r = 0; r < HL; ++r) acc[r] += ur[u][r];
                            }
                            pend += RS;
                            if (pend >= 8 * v.rounds) {
                                flush(src);
                                pend = 0;
                            }
                        }
                        flush(src);
                    }
                    if (i + 4 <= hi) {
                        const int4 ea = list4[i >> 2];
                        const int a[4] = {ea.x, ea.y, ea.z, ea.w};
                        T u4[4][HL];
#pragma unroll
                        for (int u = 0; u < 4; ++u) read_at(lb + (uint32_t)a[u], u4[u]);
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
#pragma unroll
                            for (int r = 0; r < HL; ++r) acc[r] += u4[u][r];
                        }
                        i += 4;
                    }
                    for (; i < hi; ++i) gather_one<HL, G, V4>(acc, lb + (uint32_t)list[i]);
                    flush(src);
                }
                __syncthreads();
            }
        }

        // 5. Phi of this lane's su (an update: previous Phi + entered - left),
        // P = fl32(S + Phi)
        if (x < W) {
#pragma unroll
            for (int r = 0; r < HL; ++r) {
                const int y = y0w + lrow(r);
                // the exact sums: integers times q (a power of two), or the FP64 sums
                const double a0 = INT ? sums64[0][r] * v.q : (double)accs[0][r];
                const double a1 = INT ? sums64[NSRC - 1][r] * v.q : (double)accs[NSRC - 1][r];
                double f = a0;
                if constexpr (DUAL) f = (pv[r] + a0) - a1;
                if (y < H) {
                    const size_t c = (size_t)y * v.fp + x;
                    if (v.phi) v.phi[c] = f;
                    v.P[c] = (float)(sv[r] + f);
                }
            }
        }
        if (!more) break;
        // No barrier here: every read of wave_tot, row_excl, the list and the
        // table for this strip happened before this strip's last barrier (the
        // one after the gather, or after the scan when there is no source).
        if (nitem != item) {
            if (nv.tab != v.tab) {
                load_table(nv);
                __syncthreads();
            }
            item = nitem;
            it = nit;
        }
        v = nv;
        t = nt;
        tx = ntx;
        ty = nty;
    }
    finish();
}

// ---- occupancy ----------------------------------------------------------------------

__global__ void k_occ_init(const int32_t *__restrict__ pos, int N, unsigned long long *occ, int wpr,
                           int W, unsigned long long *ctr)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int p = i < (size_t)N ? pos[i] : -1;
    if (p >= 0) {
        const int y = p / W, x = p - y * W;
        atomicOr(&occ[(size_t)y * wpr + (x >> 6)], 1ull << (x & 63));
    }
    block_sum_add(p >= 0 ? 1u : 0u, ctr, kLive);
}

// Occupancy bitmap of a caller's position list (the stateless superposition):
// the bit of su p is set for every entry 0 <= p < nsu; other entries (-1 for
// an absent pedestrian, or out of range) set nothing.
__global__ void k_occ_mark(const int32_t *__restrict__ pos, int n, unsigned long long *occ,
                           int wpr, int W, int nsu)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)n) return;
    const int p = pos[i];
    if (p < 0 || p >= nsu) return;
    const int y = p / W, x = p - y * W;
    atomicOr(&occ[(size_t)y * wpr + (x >> 6)], 1ull << (x & 63));
}

// The law's strengths over one octant of the window, (i, j) with
// 0 <= j <= i <= R at index i(i+1)/2 + j, travel as kernel arguments in
// chunks (no host buffer outlives the call that launches them).
constexpr int kOctChunk = 960;
struct OctChunk {
    int first, count;
    float v[kOctChunk];
};

// Stamp table of the gather (column-major, zero padded; FP32 strengths held
// as doubles, elem = 8, or as integers in units of q, elem = 4) from octant
// strengths: entry (dx, dy) takes the strength of (max(|dx|,|dy|),
// min(|dx|,|dy|)) for 0 < |d|_inf <= R and 0 elsewhere.  A launch writes the
// entries whose octant index is in its chunk; the launch of the first chunk
// also writes the zeros.
__global__ void k_stamp_fill(void *__restrict__ tabv, int elem, double q, int n, int ncols,
                             int stride, int padx, int pady, int R, OctChunk c)
{
    double *tab = static_cast<double *>(tabv);
    int *tabi = static_cast<int *>(tabv);
    for (int e = (int)(blockIdx.x * blockDim.x + threadIdx.x); e < n;
         e += (int)(gridDim.x * blockDim.x)) {
        const int ci = e / stride, ri = e - ci * stride;
        const int ax = abs(ci - padx), ay = abs(ri - pady);
        const int i = max(ax, ay), j = min(ax, ay);
        if (ci >= ncols || i == 0 || i > R) {
            if (c.first == 0) {
                if (elem == 4)
                    tabi[e] = 0;
                else
                    tab[e] = 0.0;
            }
            continue;
        }
        const int idx = i * (i + 1) / 2 + j - c.first;
        if (idx >= 0 && idx < c.count) {
            if (elem == 4)
                tabi[e] = (int)((double)c.v[idx] / q);  // an exact integer
            else
                tab[e] = (double)c.v[idx];
        }
    }
}

// ---- small-radius field: dense stencil over the occupancy bits -------------------
//
// With a small window and a dense crowd most of the gather's adds are the zero
// padding of its stamp.  This kernel walks the (2R+1)^2 offsets of every su
// instead.  Lane l owns column X0 + l of a 64-column tile and HL consecutive
// rows; per window row it cuts its 2R+1 occupancy bits out of the row's three
// words around the tile (the same words for the whole wave) and per offset
// adds phi when the bit is set, as acc = fma(bit, phi, acc) in FP64 with phi
// the stamp's value (uniform across the wave, held in vector registers).  The
// sum is exact, as in the gather, so both kernels give the same field bit for
// bit.

constexpr int kDenseHL = 8;       // rows per lane
constexpr int kDenseWaves = 4;    // waves per workgroup (tile: 64 x 32 su)

template <int R>
__global__ __launch_bounds__(kDenseWaves * 64) void k_field_dense(SceneView one, int n_tiles)
{
    constexpr int K = 2 * R + 1, NR = kDenseHL + 2 * R;
    const int W = one.W, H = one.H, wpr = one.wpr, fp = one.fp;
    const gptr<const unsigned long long> occ = to_global((const unsigned long long *)one.occ);
    const gptr<const double> S = to_global(one.S);
    const gptr<float> P = to_global(one.P);
    const gptr<double> phi_out = to_global(one.phi);
    const gptr<const double> tab = to_global(one.tab);
    const int lane = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    // phi(dx, dy) from the stamp: entry (dx + padx) * stride + dy + pady
    double phi[K][K];
    const int base = opaque_lane((one.padx - R) * one.stride + one.pady - R);
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = 0; b < K; ++b) phi[a][b] = tab[base + a * one.stride + b];
    const int tiles_x = (W + 63) >> 6;
    // the tile's window rows: 3 bitmap words (columns X0 - 64 .. X0 + 127) of
    // rows Y0 - R .. Y0 + TH + R - 1, staged by the whole workgroup at once
    constexpr int TH = kDenseWaves * kDenseHL, TR = TH + 2 * R;
    __shared__ unsigned long long rows[TR][3];
    const int tid = (int)threadIdx.x;
    for (int t = (int)blockIdx.x; t < n_tiles; t += (int)gridDim.x) {
        const int ty = t / tiles_x, tx = t - ty * tiles_x;
        const int x = tx * 64 + lane;
        const int Y0 = ty * TH, y0 = Y0 + wv * kDenseHL;
        // S of this lane's su, requested first: its round trip overlaps the
        // staging of the rows
        double sv[kDenseHL];
#pragma unroll
        for (int h = 0; h < kDenseHL; ++h) {
            const int y = y0 + h;
            sv[h] = S[(size_t)min(y, H - 1) * fp + min(x, W - 1)];
        }
        for (int k = tid; k < TR * 3; k += kDenseWaves * 64) {
            const int r = k / 3, c = k - r * 3;
            int sy = Y0 - R + r;
            unsigned long long wd = 0ull;
            if (one.periodic) {
                sy += sy < 0 ? H : (sy >= H ? -H : 0);
                wd = wrapped_word(occ + (size_t)sy * wpr, tx - 1 + c, W, wpr);
            } else if (sy >= 0 && sy < H && tx - 1 + c >= 0 && tx - 1 + c < wpr) {
                wd = occ[(size_t)sy * wpr + tx - 1 + c];
            }
            rows[r][c] = wd;
        }
        __syncthreads();
        if (y0 < H) {  // uniform across the wave
            double acc[kDenseHL];
#pragma unroll
            for (int h = 0; h < kDenseHL; ++h) acc[h] = 0.0;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const unsigned long long wl = rows[wv * kDenseHL + r][0];
                const unsigned long long wc = rows[wv * kDenseHL + r][1];
                const unsigned long long wr = rows[wv * kDenseHL + r][2];
                // bits of columns x - R .. x + R: from bit 64 + lane - R of wl:wc:wr
                const int p = 64 + lane - R;
                unsigned long long win;
                if (p < 64)
                    win = (wl >> p) | (wc << (64 - p));  // p >= 64 - R > 0
                else if (p == 64)
                    win = wc;
                else
                    win = (wc >> (p - 64)) | (wr << (128 - p));
#pragma unroll
                for (int i = 0; i < K; ++i) {  // source column x - R + i
                    const double bit = (double)(unsigned int)((win >> i) & 1ull);
#pragma unroll
                    for (int h = 0; h < kDenseHL; ++h) {
                        const int dy = h + R - r;  // output row y0 + h minus source row
                        if (dy >= -R && dy <= R)
                            acc[h] = fma(bit, phi[2 * R - i][dy + R], acc[h]);
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < kDenseHL; ++h) {
                const int y = y0 + h;
                if (x < W && y < H) {
                    const size_t c = (size_t)y * fp + x;
                    if (one.phi) phi_out[c] = acc[h];
                    P[c] = (float)(sv[h] + acc[h]);
                }
            }
        }
        __syncthreads();  // the rows are restaged for the next tile
    }
}

// ---- the paper's own field path: 8 sects, fan-out terms, K slots -----------------------
//
// Section 3.1 (s-1) keeps an su's strengths in 8 sects and Algorithm 3 (Eq. 1)
// sums its 8*SF fan-out terms in K blocks of m consecutive terms, each block
// into one FP32 slot, then the slots.  Here every su walks the scene's term
// list (offset, strength, sect) in that order: a term adds its strength when
// the su at the offset's source holds a pedestrian.  Lane l owns column X0 + l
// of a 64-column tile and kSectHL rows; the term is uniform across the wave
// (a scalar load), and the lane takes the source bits of its kSectHL rows
// from a column word of the source column: the workgroup stages the window's
// bitmap rows in LDS, each wave transposes them into one 128-bit word per
// column (bit j = row Y0w - R + j), and a term reads the column x - dx at bit
// R - dy.  The FP32 adds follow the term order exactly, so the field is the
// one the FP32 sums of Algorithm 3 give, bit for bit.  UPDATE: the sources are
// the su entered (+) and left (-) this tick and the sums are added to the kept
// FP32 field and image.  IMAGE: sect s of each su (its terms' FP32 sum) is
// written to plane s.

constexpr int kSectHL = 8;     // rows per lane
constexpr int kSectWaves = 4;  // waves per workgroup (tile: 64 x 32 su)
constexpr int kSectMaxR = 48;  // column words hold kSectHL + 2R <= 128 rows

template <bool UPDATE, bool IMAGE, bool SECTACC>
__global__ __launch_bounds__(kSectWaves * 64) void k_field_sect(SectView v, int n_tiles)
{
    constexpr int TH = kSectWaves * kSectHL;
    constexpr int NSRC = UPDATE ? 2 : 1;
    constexpr int MAXR = TH + 2 * kSectMaxR;   // staged rows
    constexpr int MAXC = 64 + 2 * kSectMaxR;   // columns of a wave's window
    __shared__ unsigned long long rows[NSRC][MAXR][4];
    // one spare column: a term at bit 96 reads the word after its column's last
    __shared__ uint4 cols[NSRC][kSectWaves][MAXC + 1];
    const int W = v.W, H = v.H, wpr = v.wpr, R = v.R;
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tiles_x = (W + 63) >> 6;
    const int TR = TH + 2 * R, NC = 64 + 2 * R;
    const gptr<const double> S = to_global(v.S);
    const gptr<float> P = to_global(v.P);
    const gptr<float> F = to_global(v.phi32);
    const gptr<float> img = to_global(v.image);
    const size_t plane = (size_t)W * H;
    for (int t = (int)blockIdx.x; t < n_tiles; t += (int)gridDim.x) {
        const int ty = t / tiles_x, tx = t - ty * tiles_x;
        const int X0 = tx * 64, Y0 = ty * TH, y0 = Y0 + wv * kSectHL, x = X0 + lane;
        const int wa = (X0 - R) >> 6;  // first staged word (floor)
        // 1. stage the bitmap rows Y0 - R .. Y0 + TH + R - 1, words wa .. wa + 3
        for (int k = tid; k < NSRC * TR * 4; k += kSectWaves * 64) {
            const int src = k / (TR * 4), rk = k - src * TR * 4;
            const int r = rk >> 2, c = rk & 3;
            const gptr<const unsigned long long> bits = to_global(src ? v.src2 : v.src);
            int sy = Y0 - R + r;
            const int w = wa + c;
            unsigned long long wd = 0ull;
            if (v.periodic) {
                sy = ((sy % H) + H) % H;
                wd = wrapped_word(bits + (size_t)sy * wpr, w, W, wpr);
            } else if (sy >= 0 && sy < H && w >= 0 && w < wpr) {
                wd = bits[(size_t)sy * wpr + w];
            }
            rows[src][r][c] = wd;
        }
        __syncthreads();
        // 2. this wave's column words: column X0 - R + j (j < NC), bit i = row
        // y0 - R + i (i < kSectHL + 2R)
        for (int j = lane; j < NC; j += 64) {
            const int cx = X0 - R + j, wi = (cx >> 6) - wa, b = cx & 63;
#pragma unroll
            for (int src = 0; src < NSRC; ++src) {
                unsigned int cw[4] = {0u, 0u, 0u, 0u};
                for (int i = 0; i < kSectHL + 2 * R; ++i) {
                    const unsigned int bit =
                        (unsigned int)(rows[src][wv * kSectHL + i][wi] >> b) & 1u;
                    cw[i >> 5] |= bit << (i & 31);
                }
                cols[src][wv][j] = make_uint4(cw[0], cw[1], cw[2], cw[3]);
            }
        }
        __syncthreads();
        // S (and, for an update, the kept field) of this lane's su
        double sv[kSectHL];
        float fv[kSectHL];
#pragma unroll
        for (int h = 0; h < kSectHL; ++h) {
            const size_t c = (size_t)min(y0 + h, H - 1) * v.fp + min(x, W - 1);
            sv[h] = S[c];
            fv[h] = UPDATE ? F[c] : 0.0f;
        }
        // 3. the terms in order, block by block
        float tot[kSectHL], sec[kSectHL];
#pragma unroll
        for (int h = 0; h < kSectHL; ++h) tot[h] = sec[h] = 0.0f;
        const uint32_t cbase = (uint32_t)(uintptr_t)(lds_ptr<uint4>)&cols[0][wv][0];
        const uint32_t cbase2 = (uint32_t)(uintptr_t)(lds_ptr<uint4>)&cols[NSRC - 1][wv][0];
        const bool store = x < W && y0 < H;
        for (int j = 0; j < v.K; ++j) {
            float blk[kSectHL];
#pragma unroll
            for (int h = 0; h < kSectHL; ++h) blk[h] = 0.0f;
            const int i1 = min(j * v.m + v.m, v.n_real);
            for (int i = j * v.m; i < i1; ++i) {
                const int2 term = v.terms[i];
                const int info = __builtin_amdgcn_readfirstlane(term.x);
                const float ph = __int_as_float(__builtin_amdgcn_readfirstlane(term.y));
                const int dx = (info & 0xFF) - 128, dy = ((info >> 8) & 0xFF) - 128;
                // bits R - dy .. R - dy + 7 of column x - dx
                const int sh = R - dy, q = sh >> 5, rr = sh & 31;
                const uint32_t off = (uint32_t)((lane + R - dx) * 16 + q * 4);
                typedef const __attribute__((address_space(3))) unsigned int *lds_u;
                const lds_u a = reinterpret_cast<lds_u>(cbase + off);
                unsigned int bits = __builtin_amdgcn_alignbit(a[1], a[0], rr);
                unsigned int bits2 = 0u;
                if constexpr (UPDATE) {
                    const lds_u a2 = reinterpret_cast<lds_u>(cbase2 + off);
                    bits2 = __builtin_amdgcn_alignbit(a2[1], a2[0], rr);
                }
#pragma unroll
                for (int h = 0; h < kSectHL; ++h) {
                    float d = (float)((bits >> h) & 1u);
                    if constexpr (UPDATE) d -= (float)((bits2 >> h) & 1u);
                    blk[h] = fmaf(d, ph, blk[h]);
                    if constexpr (SECTACC) sec[h] = fmaf(d, ph, sec[h]);
                }
                if constexpr (IMAGE && SECTACC) {
                    if (info & (1 << 20)) {  // the last term of its sect
                        const int s = (info >> 16) & 7;
#pragma unroll
                        for (int h = 0; h < kSectHL; ++h) {
                            const size_t c = (size_t)(y0 + h) * W + x;
                            if (store && y0 + h < H)
                                img[s * plane + c] = UPDATE ? img[s * plane + c] + sec[h] : sec[h];
                            sec[h] = 0.0f;
                        }
                    }
                }
            }
            if constexpr (IMAGE && !SECTACC) {  // K = 8: block j is sect j
#pragma unroll
                for (int h = 0; h < kSectHL; ++h) {
                    const size_t c = (size_t)(y0 + h) * W + x;
                    if (store && y0 + h < H)
                        img[j * plane + c] = UPDATE ? img[j * plane + c] + blk[h] : blk[h];
                }
            }
#pragma unroll
            for (int h = 0; h < kSectHL; ++h) tot[h] = tot[h] + blk[h];
        }
        if constexpr (IMAGE) {
            if (v.n_real == 0 && !UPDATE) {  // R = 0: no terms, every sect is 0
                for (int s = 0; s < 8; ++s)
#pragma unroll
                    for (int h = 0; h < kSectHL; ++h)
                        if (store && y0 + h < H) img[s * plane + (size_t)(y0 + h) * W + x] = 0.0f;
            }
        }
        // 4. the FP32 field (an update adds its sum to the kept field) and P
#pragma unroll
        for (int h = 0; h < kSectHL; ++h) {
            if (store && y0 + h < H) {
                const size_t c = (size_t)(y0 + h) * v.fp + x;
                const float f = UPDATE ? fv[h] + tot[h] : tot[h];
                F[c] = f;
                P[c] = (float)(sv[h] + (double)f);
            }
        }
        __syncthreads();  // rows and columns are restaged for the next tile
    }
}

// ---- decide + claim (k-2, k-3 registration) --------------------------------------------
//
// One thread per pedestrian (internal id i, ids ordered by position at
// creation, so a wave's pedestrians are close together and share cache
// lines).  Its loads are independent and issued together: the occupancy bits
// of the three rows around it (one bitmap word per row, and the neighbouring
// word when it stands at a word edge) and the field at the 9 candidate su.
// Then the decision, the election key and the claim (an atomic minimum on
// the target's claim word).  Pedestrians that have left are skipped (the
// commit kernel clears their outputs).

constexpr int kDecideThreads = 256;

// Commit workgroup size: 256 threads for one scene, 128 in a batch, whose
// launch covers many small scenes (measured: a 96-scene ensemble tick
// 1.80 -> 1.75 ms with 128; single scenes gain nothing from it)
template <bool MULTI>
__host__ __device__ constexpr int commit_threads()
{
    return MULTI ? 128 : 256;
}

// workgroups of one scene's decide launch (at least one: it also clears the
// moved-su bitmaps)
__host__ __device__ constexpr int decide_block_count(int N)
{
    return N > 0 ? (N + kDecideThreads - 1) / kDecideThreads : 1;
}

// The view of this workgroup's scene: views[block_scene[block]] (MULTI) or
// the kernel argument `one`.
template <bool MULTI>
__device__ __forceinline__ const SceneView &block_view(const SceneView &one,
                                                       const SceneView *__restrict__ views,
                                                       const int32_t *__restrict__ block_scene)
{
    if constexpr (MULTI) return views[block_scene[blockIdx.x]];
    return one;
}

template <bool MULTI>
__global__ __launch_bounds__(kDecideThreads) void k_decide_claim(
    SceneView one, const SceneView *__restrict__ views, const int32_t *__restrict__ block_scene)
{
    const SceneView &v = block_view<MULTI>(one, views, block_scene);
    const int W = v.W, H = v.H, wpr = v.wpr, N = v.N;
    const int lb = (int)blockIdx.x - v.dec_block0;
    const int i = lb * kDecideThreads + (int)threadIdx.x;
    const gptr<const unsigned long long> occ = to_global((const unsigned long long *)v.occ);
    const gptr<const float> P = to_global((const float *)v.P);
    const gptr<ClaimRec> claims = to_global(v.claims);
    const gptr<unsigned long long> key = to_global(v.key), ctr = to_global(v.ctr);
    const gptr<int32_t> target = to_global(v.target);
    const gptr<uint8_t> flags = to_global(v.flags);
    if (v.moved_from) {
        // the previous tick's moves have been applied to the field
        const int nb = decide_block_count(N);
        const size_t nwd = (size_t)wpr * H;
        for (size_t k = (size_t)lb * kDecideThreads + threadIdx.x; k < nwd;
             k += (size_t)nb * kDecideThreads) {
            to_global(v.moved_from)[k] = 0ull;
            to_global(v.moved_to)[k] = 0ull;
        }
    }
    const unsigned long long seed = v.seed;
    const float phi_axial = v.phi_axial, phi_diag = v.phi_diag;
    unsigned int movers = 0, ties = 0;
    // the step index and this pedestrian's arrays are requested together and
    // waited for once (the empty asm takes all of them, so no load is moved
    // behind a branch that would wait for it alone)
    unsigned long long t = ctr[0];
    int p = -1, h = 0;
    uint32_t eid = 0;
    unsigned int wp = 1u;
    if (i < N) {
        p = to_global((const int32_t *)v.pos)[i];
        eid = (uint32_t)to_global((const int32_t *)v.ext)[i];
        if (v.heading) h = (int)to_global(v.heading)[i];
        if (v.walk) wp = (unsigned int)to_global(v.walk)[i];
    }
    asm volatile("" : "+v"(p), "+v"(eid), "+v"(h), "+v"(wp), "+v"(t));
    if (p >= 0) {
        if (wp > 1u && (t + eid) % wp != 0ull) {
            // resting this tick: stays, registers for nothing
            target[i] = p;
            flags[i] = 0;
        } else {
            const int y = p / W, x = p - y * W;
            // occupancy of columns x - 1, x, x + 1 in rows y - 1, y, y + 1: bit
            // (dx + 1) of nb3[dy + 1]; the field there in pv (+inf on obstacle su
            // and outside a bounded grid); their rows and columns in row[] and
            // col[] (periodic: wrapped across the edges)
            unsigned int nb3[3];
            float pv[3][3];
            // bounded grids of a single scene: the 5 x 5 block of centres
            // around the pedestrian (solo_ok once it is loaded).  Tori and
            // batches register every move: in a batch, decide runs beside the
            // other radius groups' field launches, and the lighter decide and
            // commit measured slower there (256-scene tick 3.39 -> 3.48 ms:
            // the concurrent schedule of the groups shifted against the field
            // of the largest stamps)
            unsigned int win25 = 0u;
            bool solo_ok = false;
            int col[3], row[3];
            if (v.periodic && W >= 3 && wpr >= 2) {
                col[0] = x == 0 ? W - 1 : x - 1;
                col[1] = x;
                col[2] = x == W - 1 ? 0 : x + 1;
                // per row, issued unconditionally and waited for once: the
                // three field values from column xb0 (x - 1 clamped into
                // [0, W - 3]), the bitmap word pair from word wp0 (holding
                // column x and the word on the side of x's nearer word edge),
                // and the field value and bitmap word of column xs, the
                // neighbour across the seam of a lane at x = 0 or W - 1
                const int w = x >> 6, b = x & 63;
                const int xb0 = min(max(x - 1, 0), W - 3);
                const int wp0 = min(max(b < 32 ? w - 1 : w, 0), wpr - 2);
                const int xs = x == 0 ? W - 1 : 0, ws = xs >> 6;
                unsigned long long q0[3], q1[3], qs[3];
                float t0[3], t1[3], t2[3], ts[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    int yy = y - 1 + r;
                    yy += yy < 0 ? H : (yy >= H ? -H : 0);
                    row[r] = yy;
                    const size_t rw = (size_t)yy * wpr;
                    q0[r] = occ[rw + wp0];
                    q1[r] = occ[rw + wp0 + 1];
                    qs[r] = occ[rw + ws];
                    const size_t rp = (size_t)yy * v.fp;
                    t0[r] = P[rp + xb0];
                    t1[r] = P[rp + xb0 + 1];
                    t2[r] = P[rp + xb0 + 2];
                    ts[r] = P[rp + xs];
                }
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    asm volatile("" : "+v"(q0[r]), "+v"(q1[r]), "+v"(qs[r]));
                    asm volatile("" : "+v"(t0[r]), "+v"(t1[r]), "+v"(t2[r]), "+v"(ts[r]));
                }
                const bool mid_first = wp0 == w;
                const int sh = x - 1 - xb0;  // -1 at x = 0, +1 at x = W - 1, else 0
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const unsigned long long mid = mid_first ? q0[r] : q1[r];
                    // the pair's other word: w - 1 when b = 0 < x, w + 1 when
                    // b = 63 and x < W - 1
                    const unsigned long long oth = mid_first ? q1[r] : q0[r];
                    const unsigned int cl =
                        x == 0 ? (unsigned int)(qs[r] >> (xs & 63)) & 1u
                               : (b > 0 ? (unsigned int)(mid >> (b - 1)) & 1u
                                        : (unsigned int)(oth >> 63));
                    const unsigned int cc = (unsigned int)(mid >> b) & 1u;
                    const unsigned int cr =
                        x == W - 1 ? (unsigned int)qs[r] & 1u
                                   : (b < 63 ? (unsigned int)(mid >> (b + 1)) & 1u
                                             : (unsigned int)oth & 1u);
                    nb3[r] = cl | (cc << 1) | (cr << 2);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int k = c + sh;
                        const float tv = k <= 0 ? t0[r] : (k == 1 ? t1[r] : t2[r]);
                        pv[r][c] = (c == 0 && x == 0) || (c == 2 && x == W - 1) ? ts[r] : tv;
                    }
                }
            } else if (v.periodic) {
                // tori narrower than 3 su or one bitmap word
                col[0] = x == 0 ? W - 1 : x - 1;
                col[1] = x;
                col[2] = x == W - 1 ? 0 : x + 1;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    int yy = y - 1 + r;
                    yy += yy < 0 ? H : (yy >= H ? -H : 0);
                    row[r] = yy;
                    const size_t rw = (size_t)yy * wpr;
                    unsigned int m = 0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        m |= (unsigned int)(occ[rw + (col[c] >> 6)] >> (col[c] & 63) & 1ull) << c;
                        pv[r][c] = P[(size_t)yy * v.fp + col[c]];
                    }
                    nb3[r] = m;
                }
            } else {
                const int w = x >> 6, b = x & 63;
                col[0] = x - 1;
                col[1] = x;
                col[2] = x + 1;
                // every load is issued unconditionally at a clamped (in-grid)
                // su and all are waited for once; the values outside the grid
                // or beside the word are then replaced
                // per row the word of column x and the word on the side of x's
                // nearer word edge (the only neighbour word a column x - 1 or
                // x + 1 can fall into)
                // (one scene: rows y - 2 and y + 2 too, the 5 x 5 block of
                // centres that tells whether anyone else can register at the
                // chosen target)
                constexpr bool SOLO = !MULTI;
                unsigned long long wm[5] = {}, we[5] = {};
                float pr[3][3];
                const int wn = min(max(b < 32 ? w - 1 : w + 1, 0), wpr - 1);
#pragma unroll
                for (int r = 0; r < 5; ++r) {
                    if (!SOLO && (r == 0 || r == 4)) continue;
                    const int yc = min(max(y - 2 + r, 0), H - 1);
                    const size_t rw = (size_t)yc * wpr;
                    wm[r] = occ[rw + w];
                    we[r] = occ[rw + wn];
                    if (r >= 1 && r <= 3) {
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            pr[r - 1][c] = P[(size_t)yc * v.fp + min(max(x - 1 + c, 0), W - 1)];
                    }
                }
#pragma unroll
                for (int r = 0; r < 5; ++r)
                    if (SOLO || (r >= 1 && r <= 3)) asm volatile("" : "+v"(wm[r]), "+v"(we[r]));
#pragma unroll
                for (int r = 0; r < 3; ++r)
                    asm volatile("" : "+v"(pr[r][0]), "+v"(pr[r][1]), "+v"(pr[r][2]));
                // centres in columns x - 2 .. x + 2 of rows y - 2 .. y + 2: bit
                // 5r + c of win25 is column x - 2 + c of row y - 2 + r (0 outside
                // the grid; the word beside x's nearer word edge holds every such
                // column off word w)
#pragma unroll
                for (int r = 0; r < 5 && SOLO; ++r) {
                    const int yy = y - 2 + r;
                    unsigned long long lo, hi;
                    int at;
                    if (b < 32) {
                        lo = w > 0 ? we[r] : 0ull;
                        hi = wm[r];
                        at = 62 + b;
                    } else {
                        lo = wm[r];
                        hi = w + 1 < wpr ? we[r] : 0ull;
                        at = b - 2;
                    }
                    const unsigned long long bits =
                        at >= 64 ? hi >> (at - 64) : (lo >> at) | (hi << (64 - at));
                    if (yy >= 0 && yy < H) win25 |= ((unsigned int)bits & 31u) << (5 * r);
                }
                solo_ok = SOLO;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const int yy = y - 1 + r;
                    row[r] = yy;
                    const bool row_in = yy >= 0 && yy < H;
                    const unsigned long long mid = row_in ? wm[r + 1] : 0ull;
                    const unsigned long long lft =
                        row_in && b == 0 && w > 0 ? we[r + 1] : 0ull;
                    const unsigned long long rgt =
                        row_in && b == 63 && w + 1 < wpr ? we[r + 1] : 0ull;
                    const unsigned int cl = b > 0 ? (unsigned int)(mid >> (b - 1)) & 1u
                                                  : (unsigned int)(lft >> 63);
                    const unsigned int cc = (unsigned int)(mid >> b) & 1u;
                    const unsigned int cr = b < 63 ? (unsigned int)(mid >> (b + 1)) & 1u
                                                   : (unsigned int)rgt & 1u;
                    nb3[r] = cl | (cc << 1) | (cr << 2);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int xx = x - 1 + c;
                        pv[r][c] = row_in && xx >= 0 && xx < W ? pr[r][c] : INFINITY;
                    }
                }
            }
            // heading term of move d: -w_h cos(45 deg * turn), turn = 0..4
            const float hw_axis = v.hw_axis, hw_diag = v.hw_diag;
            auto heading_term = [&](int d) -> float {
                if (h == 0) return 0.0f;
                int turn = h > d ? h - d : d - h;
                turn = turn > 4 ? 8 - turn : turn;
                return turn == 0 ? -hw_axis
                                 : turn == 1 ? -hw_diag
                                             : turn == 2 ? 0.0f : turn == 3 ? hw_diag : hw_axis;
            };
            float lo = pv[1][1], lo2 = INFINITY;
            int best = 0;
#pragma unroll
            for (int d = 1; d <= 8; ++d) {
                const int r = 1 + kDirY[d], c = 1 + kDirX[d];
                const float pc = pv[r][c];
                if (!((nb3[r] >> c) & 1u) && pc < INFINITY) {
                    const float u = (pc - ((d & 1) ? phi_axial : phi_diag)) + heading_term(d);
                    if (u < lo) {
                        lo2 = lo;
                        lo = u;
                        best = d;
                    } else if (u < lo2) {
                        lo2 = u;
                    }
                }
            }
            const float scale = fmaxf(fmaxf(fabsf(lo), fabsf(lo2)), 1.0f);
            const bool tied = lo2 < INFINITY && (lo2 - lo) <= 1e-5f * scale;
            int tgt = p;
            bool mover = false, solo = false;
            if (best != 0) {
                tgt = row[1 + kDirY[best]] * W + col[1 + kDirX[best]];
                const uint32_t r = philox_w0(eid, (uint32_t)t, (uint32_t)(t >> 32), 0u,
                                             (uint32_t)seed, (uint32_t)(seed >> 32));
                const unsigned long long kk = ((unsigned long long)r << 32) | eid;
                // Only a pedestrian on one of the 8 su around the target can
                // register there (moves reach the 8 neighbours).  With none
                // but this one, it is the election's only registrant and wins
                // (the smallest key of one): no claim is needed.
                if (solo_ok) {
                    const int dx = kDirX[best], dy = kDirY[best];
                    const unsigned int m = 7u << (dx + 1);
                    const unsigned int around = (m | (m << 5) | (m << 10)) << (5 * (dy + 1));
                    solo = (win25 & around & ~(1u << 12)) == 0u;  // bit 12: this pedestrian
                }
                if (!solo) {
                    __hip_atomic_fetch_min(&claims[tgt].word, kk, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    // one more registration at the target (s-2: at most 8 under
                    // v_max = 1); the count is read by the election's winner in
                    // commit, so this atomic returns nothing and nothing waits
                    __hip_atomic_fetch_add(&claims[tgt].regs, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
                key[i] = kk;
                mover = true;
            }
            target[i] = tgt;
            flags[i] = (uint8_t)((mover ? kFlagMover : 0u) | (tied ? kFlagTied : 0u) |
                                 (solo ? kFlagSolo : 0u));
            movers += mover;
            ties += tied;
        }
    }
    block_sums_add<2>({(int)movers, (int)ties}, ctr, {kMovers, kTied});
}

// ---- commit (k-4 moves, exits) -------------------------------------------------------

template <bool MULTI>
__global__ __launch_bounds__(commit_threads<MULTI>()) void k_commit(SceneView one,
                                                           const SceneView *__restrict__ views,
                                                           const int32_t *__restrict__ block_scene)
{
    const SceneView &v = block_view<MULTI>(one, views, block_scene);
    const int lb = (int)blockIdx.x - v.com_block0;
    const int i = lb * commit_threads<MULTI>() + (int)threadIdx.x;
    const int W = v.W, wpr = v.wpr;
    const gptr<int32_t> pos = to_global(v.pos), target = to_global(v.target);
    const gptr<uint8_t> flags = to_global(v.flags);
    const gptr<const uint8_t> exitm = to_global(v.exitm);
    const gptr<const unsigned long long> key = to_global((const unsigned long long *)v.key);
    const gptr<ClaimRec> claims = to_global(v.claims);
    const gptr<unsigned long long> occ = to_global(v.occ), ctr = to_global(v.ctr);
    bool was_live = false, won = false, left = false;
    unsigned int regs_seen = 0;  // registrants of the su this thread won
    if (i < v.N) {
        // independent loads first (one round trip), then, for movers, the
        // claim word, the exit flag, the registration count and the mover's
        // own key together
        const int p = pos[i];
        const uint8_t f = flags[i];
        const int tgt = target[i];
        if (p < 0) {
            target[i] = -1;
            flags[i] = 0;
        } else {
            was_live = true;
            if (f & kFlagMover) {
                bool win;
                bool to_exit;
                if (f & kFlagSolo) {
                    // the target's only possible registrant (decide saw no
                    // other pedestrian around it) wins without a claim
                    win = true;
                    regs_seen = 1u;
                    to_exit = exitm[tgt] != 0;
                } else {
                    // the winner is the only registrant that finds its own key;
                    // it also resets the word, which losers then read as "not
                    // mine"; the claim record in one 16-byte load: word,
                    // registrations
                    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
                    const u32x4 rec = *reinterpret_cast<const __attribute__((address_space(1)))
                                                            u32x4 *>(&claims[tgt]);
                    const unsigned long long cw = ((unsigned long long)rec[1] << 32) | rec[0];
                    to_exit = exitm[tgt] != 0;
                    const unsigned int nreg = rec[2];
                    const unsigned long long kk = key[i];
                    win = cw == kk;
                    if (win) {
                        // every registration of this tick is counted by now
                        // (decide has finished); each claimed su has one
                        // winner, which reads the count before it clears it
                        regs_seen = nreg;
                        claims[tgt].word = ~0ull;
                        claims[tgt].regs = 0u;
                    }
                }
                if (win) {
                    won = true;
                    const int y = p / W, x = p - y * W;
                    const size_t wp = (size_t)y * wpr + (x >> 6);
                    const unsigned long long bp = 1ull << (x & 63);
                    if (v.moved_from)
                        __hip_atomic_fetch_or(&to_global(v.moved_from)[wp], bp, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    if (to_exit) {
                        __hip_atomic_fetch_and(&occ[wp], ~bp, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        left = true;
                        pos[i] = -1;
                    } else {
                        const int ty = tgt / W, tx = tgt - ty * W;
                        const size_t wt = (size_t)ty * wpr + (tx >> 6);
                        const unsigned long long bt = 1ull << (tx & 63);
                        if (wt == wp) {
                            // one word: the bit of p is set and the bit of the
                            // target clear (it was a free candidate, and this
                            // winner is the only one to enter it), so one
                            // exclusive or moves the pedestrian
                            __hip_atomic_fetch_xor(&occ[wp], bp | bt, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                        } else {
                            __hip_atomic_fetch_and(&occ[wp], ~bp, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                            __hip_atomic_fetch_or(&occ[wt], bt, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                        }
                        if (v.moved_to)
                            __hip_atomic_fetch_or(&to_global(v.moved_to)[wt], 1ull << (tx & 63),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        pos[i] = tgt;
                    }
                    flags[i] = f | kFlagWon;
                }
            }
        }
    }
    if (lb == 0 && threadIdx.x == 0)
        __hip_atomic_fetch_add(&ctr[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wave_max_into(regs_seen, ctr, kMaxClaim);
    block_sums_add<4>({was_live ? 1 : 0, won ? 1 : 0, left ? 1 : 0, left ? -1 : 0}, ctr,
                      {kPedSteps, kMoved, kEvacuated, kLive});
}

// ---- pedestrians larger than one su (section 2; Table VI) -----------------------------
//
// A pedestrian covers the (2a+1) x (2b+1) block of su centred on its su.  The
// bitmap `bodies` holds every covered su; `occ` keeps the centres, the field's
// sources.  A move e is a candidate when the su the shifted body enters are in
// the grid (or wrap), off obstacles and off other bodies; a mover registers
// (claim word, registration count) at each of them and wins if its key is the
// smallest at all of them; the smallest key's holder at an su clears that su's
// claim word after it has read all of its own, so a later reader finds either
// that key or the cleared word, never its own.  A winner whose shifted body
// covers an exit su leaves.

constexpr int kBodyMaxHalf = 7;  // bodies up to 15 x 15 su

// One step of the body of half-widths (a, b) at (x, y) by (ex, ey): the su it
// enters (shifted body minus current body), or with `trailing` the su it
// leaves (current body minus shifted body), as unwrapped coordinates handed to
// f(sx, sy).  A column of 2b+1 su when ex != 0, a row of 2a+1 su when ey != 0,
// their shared corner once.
template <typename F>
__device__ __forceinline__ void body_edge(int x, int y, int a, int b, int ex, int ey,
                                          bool trailing, F f)
{
    // entered: column x + ex(a+1) over rows y + ey + j; row y + ey(b+1) over
    // columns x + ex + i.  Leaving: column x - ex a over rows y + j; row
    // y - ey b over columns x + i.
    const int cx = trailing ? x - ex * a : x + ex * (a + 1);
    const int ry = trailing ? y - ey * b : y + ey * (b + 1);
    const int oy = trailing ? 0 : ey, ox = trailing ? 0 : ex;
    if (ex != 0)
        for (int j = -b; j <= b; ++j) f(cx, y + oy + j);
    if (ey != 0)
        for (int i = -a; i <= a; ++i) {
            const int sx = x + ox + i;
            if (ex != 0 && sx == cx) continue;  // the corner, already listed
            f(sx, ry);
        }
}

// Bits of columns x0 .. x0 + n - 1 (n <= 32, unwrapped) of bitmap row `row`:
// on a torus taken modulo W (W >= 64), on a bounded grid with the columns
// outside [0, W) read as set (blocked).
__device__ __forceinline__ unsigned int row_window(gptr<const unsigned long long> row, int x0,
                                                   int n, int W, int wpr, bool periodic)
{
    const unsigned long long nmask = (1ull << n) - 1ull;
    if (periodic) {
        const int w0 = x0 >= 0 ? x0 >> 6 : -((63 - x0) >> 6);
        const int off = x0 - 64 * w0;
        unsigned long long v = wrapped_word(row, w0, W, wpr) >> off;
        if (off + n > 64) v |= wrapped_word(row, w0 + 1, W, wpr) << (64 - off);
        return (unsigned int)(v & nmask);
    }
    const int lo = max(x0, 0), hi = min(x0 + n - 1, W - 1);
    unsigned long long out = nmask;
    if (lo <= hi) {
        const int w = lo >> 6, bo = lo & 63, m = hi - lo + 1;
        unsigned long long v = row[w] >> bo;
        if (bo != 0 && w + 1 < wpr) v |= row[w + 1] << (64 - bo);
        v &= m == 64 ? ~0ull : ((1ull << m) - 1ull);
        const unsigned long long in = (m == 64 ? ~0ull : ((1ull << m) - 1ull)) << (lo - x0);
        out = (out & ~in) | (v << (lo - x0));
    }
    return (unsigned int)out;
}

__device__ __forceinline__ int wrap_or_keep(int v, int n, bool periodic)
{
    if (!periodic) return v;
    v %= n;
    return v < 0 ? v + n : v;
}

// Body bitmap from the positions: every live pedestrian sets its block.
__global__ void k_body_init(SceneView v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)v.N) return;
    const int p = v.pos[i];
    if (p < 0) return;
    const int W = v.W, H = v.H, x = p % W, y = p / W;
    const bool per = v.periodic != 0;
    for (int j = -v.bb; j <= v.bb; ++j)
        for (int q = -v.ba; q <= v.ba; ++q) {
            const int sx = wrap_or_keep(x + q, W, per), sy = wrap_or_keep(y + j, H, per);
            __hip_atomic_fetch_or(&v.bodies[(size_t)sy * v.wpr + (sx >> 6)], 1ull << (sx & 63),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
}

// Decide + claim for bodies: one thread per pedestrian.  The (2a+3) x (2b+3)
// window around the body (covered and obstacle su, blocked outside a bounded
// grid) is read row by row; a move is a candidate when the su it enters are
// all clear.  Values, tie-break, near-tie flag and keys as for one su.
__global__ __launch_bounds__(kDecideThreads) void k_decide_body(SceneView v)
{
    const int W = v.W, H = v.H, wpr = v.wpr, N = v.N;
    const int i = (int)blockIdx.x * kDecideThreads + (int)threadIdx.x;
    const bool per = v.periodic != 0;
    const int a = v.ba, b = v.bb, bw = 2 * a + 1, bh = 2 * b + 1;
    const gptr<const unsigned long long> bodies =
        to_global((const unsigned long long *)v.bodies);
    const gptr<const unsigned long long> obits = to_global(v.obits);
    const gptr<const float> P = to_global((const float *)v.P);
    const gptr<ClaimRec> claims = to_global(v.claims);
    const gptr<unsigned long long> key = to_global(v.key), ctr = to_global(v.ctr);
    if (v.moved_from) {
        const int nb = decide_block_count(N);
        const size_t nwd = (size_t)wpr * H;
        for (size_t k = (size_t)blockIdx.x * kDecideThreads + threadIdx.x; k < nwd;
             k += (size_t)nb * kDecideThreads) {
            to_global(v.moved_from)[k] = 0ull;
            to_global(v.moved_to)[k] = 0ull;
        }
    }
    const unsigned long long t = ctr[0], seed = v.seed;
    unsigned int movers = 0, ties = 0, regs_seen = 0;
    const int p = i < N ? to_global((const int32_t *)v.pos)[i] : -1;
    if (p >= 0) {
        const uint32_t eid = (uint32_t)to_global((const int32_t *)v.ext)[i];
        const int h = v.heading ? (int)to_global(v.heading)[i] : 0;
        const unsigned int wp = v.walk ? (unsigned int)to_global(v.walk)[i] : 1u;
        if (wp > 1u && (t + eid) % wp != 0ull) {
            to_global(v.target)[i] = p;
            to_global(v.flags)[i] = 0;
        } else {
            const int y = p / W, x = p - y * W;
            // window rows r = 0 .. bh + 1 (grid row y - b - 1 + r), bit c of a
            // row = column x - a - 1 + c
            unsigned int win[2 * kBodyMaxHalf + 3];
            for (int r = 0; r < bh + 2; ++r) {
                const int yy = y - b - 1 + r;
                if (!per && (yy < 0 || yy >= H)) {
                    win[r] = (1u << (bw + 2)) - 1u;
                    continue;
                }
                const size_t ro = (size_t)wrap_or_keep(yy, H, per) * wpr;
                unsigned int m = row_window(bodies + ro, x - a - 1, bw + 2, W, wpr, per);
                if (v.obits) m |= row_window(obits + ro, x - a - 1, bw + 2, W, wpr, per);
                win[r] = m;
            }
            const float phi_axial = v.phi_axial, phi_diag = v.phi_diag;
            const float hw_axis = v.hw_axis, hw_diag = v.hw_diag;
            auto heading_term = [&](int d) -> float {
                if (h == 0) return 0.0f;
                int turn = h > d ? h - d : d - h;
                turn = turn > 4 ? 8 - turn : turn;
                return turn == 0 ? -hw_axis
                                 : turn == 1 ? -hw_diag
                                             : turn == 2 ? 0.0f : turn == 3 ? hw_diag : hw_axis;
            };
            float lo = P[(size_t)y * v.fp + x], lo2 = INFINITY;
            int best = 0;
            for (int d = 1; d <= 8; ++d) {
                const int ex = kDirX[d], ey = kDirY[d];
                bool blocked = false;
                if (ex != 0) {
                    const int c = ex > 0 ? bw + 1 : 0;
                    for (int r = 1 + ey; r <= bh + ey; ++r) blocked |= (win[r] >> c) & 1u;
                }
                if (ey != 0) {
                    const unsigned int row = win[ey > 0 ? bh + 1 : 0];
                    blocked |= ((row >> (1 + ex)) & ((1u << bw) - 1u)) != 0u;
                }
                if (blocked) continue;
                const int nx = wrap_or_keep(x + ex, W, per), ny = wrap_or_keep(y + ey, H, per);
                const float pc = P[(size_t)ny * v.fp + nx];
                if (!(pc < INFINITY)) continue;
                const float u = (pc - ((d & 1) ? phi_axial : phi_diag)) + heading_term(d);
                if (u < lo) {
                    lo2 = lo;
                    lo = u;
                    best = d;
                } else if (u < lo2) {
                    lo2 = u;
                }
            }
            const float scale = fmaxf(fmaxf(fabsf(lo), fabsf(lo2)), 1.0f);
            const bool tied = lo2 < INFINITY && (lo2 - lo) <= 1e-5f * scale;
            int tgt = p;
            if (best != 0) {
                const int ex = kDirX[best], ey = kDirY[best];
                tgt = wrap_or_keep(y + ey, H, per) * W + wrap_or_keep(x + ex, W, per);
                const uint32_t r = philox_w0(eid, (uint32_t)t, (uint32_t)(t >> 32), 0u,
                                             (uint32_t)seed, (uint32_t)(seed >> 32));
                const unsigned long long kk = ((unsigned long long)r << 32) | eid;
                body_edge(x, y, a, b, ex, ey, false, [&](int sx, int sy) {
                    const size_t q = (size_t)wrap_or_keep(sy, H, per) * W + wrap_or_keep(sx, W, per);
                    __hip_atomic_fetch_min(&claims[q].word, kk, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    regs_seen = max(regs_seen, 1u + __hip_atomic_fetch_add(
                                                        &claims[q].regs, 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT));
                });
                key[i] = kk;
                ++movers;
            }
            to_global(v.target)[i] = tgt;
            to_global(v.flags)[i] =
                (uint8_t)((best != 0 ? kFlagMover : 0u) | (tied ? kFlagTied : 0u));
            ties += tied;
        }
    }
    block_sums_add<2>({(int)movers, (int)ties}, ctr, {kMovers, kTied});
    block_max_into(regs_seen, ctr, kMaxClaim);
}

// Commit for bodies: a mover reads the claim words of every su it entered; it
// won if all hold its key.  It then clears the words it holds (with their
// registration counts).  A winner clears the su it leaves and sets the su it
// enters in the body bitmap and moves its centre bit, or, when its shifted
// body covers an exit su, clears its whole body and leaves.
__global__ __launch_bounds__(256) void k_commit_body(SceneView v)
{
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    const int W = v.W, H = v.H, wpr = v.wpr;
    const bool per = v.periodic != 0;
    const int a = v.ba, b = v.bb;
    const gptr<int32_t> pos = to_global(v.pos), target = to_global(v.target);
    const gptr<uint8_t> flags = to_global(v.flags);
    const gptr<const uint8_t> exitm = to_global(v.exitm);
    const gptr<ClaimRec> claims = to_global(v.claims);
    const gptr<unsigned long long> occ = to_global(v.occ), bodies = to_global(v.bodies),
                                   ctr = to_global(v.ctr);
    bool was_live = false, won = false, left = false;
    auto su_of = [&](int sx, int sy) {
        return (size_t)wrap_or_keep(sy, H, per) * W + wrap_or_keep(sx, W, per);
    };
    auto bit_and = [&](size_t q, bool set) {
        const int qy = (int)(q / W), qx = (int)(q - (size_t)qy * W);
        const size_t wd = (size_t)qy * wpr + (qx >> 6);
        const unsigned long long m = 1ull << (qx & 63);
        if (set)
            __hip_atomic_fetch_or(&bodies[wd], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_fetch_and(&bodies[wd], ~m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    if (i < v.N) {
        const int p = pos[i];
        const uint8_t f = flags[i];
        const int tgt = target[i];
        if (p < 0) {
            target[i] = -1;
            flags[i] = 0;
        } else {
            was_live = true;
            if (f & kFlagMover) {
                const unsigned long long kk = to_global((const unsigned long long *)v.key)[i];
                const int y = p / W, x = p - y * W, ty = tgt / W, tx = tgt - ty * W;
                int ex = tx - x, ey = ty - y;
                if (per) {
                    ex = ex > 1 ? ex - W : (ex < -1 ? ex + W : ex);
                    ey = ey > 1 ? ey - H : (ey < -1 ? ey + H : ey);
                }
                // read every claim word first, then clear the ones this mover holds
                bool all_mine = true, at_exit = false;
                unsigned int held = 0u;
                int k = 0;
                body_edge(x, y, a, b, ex, ey, false, [&](int sx, int sy) {
                    const size_t q = su_of(sx, sy);
                    const bool mine = claims[q].word == kk;
                    all_mine &= mine;
                    held |= (mine ? 1u : 0u) << k;
                    at_exit |= exitm[q] != 0;
                    ++k;
                });
                k = 0;
                body_edge(x, y, a, b, ex, ey, false, [&](int sx, int sy) {
                    if ((held >> k) & 1u) {
                        const size_t q = su_of(sx, sy);
                        claims[q].word = ~0ull;
                        claims[q].regs = 0u;
                    }
                    ++k;
                });
                if (all_mine) {
                    won = true;
                    const size_t wp = (size_t)y * wpr + (x >> 6);
                    __hip_atomic_fetch_and(&occ[wp], ~(1ull << (x & 63)), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    if (v.moved_from)
                        __hip_atomic_fetch_or(&to_global(v.moved_from)[wp], 1ull << (x & 63),
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (at_exit) {
                        left = true;
                        for (int j = -b; j <= b; ++j)
                            for (int q = -a; q <= a; ++q) bit_and(su_of(x + q, y + j), false);
                        pos[i] = -1;
                    } else {
                        body_edge(x, y, a, b, ex, ey, true,
                                  [&](int sx, int sy) { bit_and(su_of(sx, sy), false); });
                        body_edge(x, y, a, b, ex, ey, false,
                                  [&](int sx, int sy) { bit_and(su_of(sx, sy), true); });
                        const size_t wt = (size_t)ty * wpr + (tx >> 6);
                        __hip_atomic_fetch_or(&occ[wt], 1ull << (tx & 63), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                        if (v.moved_to)
                            __hip_atomic_fetch_or(&to_global(v.moved_to)[wt], 1ull << (tx & 63),
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        pos[i] = tgt;
                    }
                    flags[i] = f | kFlagWon;
                }
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_fetch_add(&ctr[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    block_sums_add<4>({was_live ? 1 : 0, won ? 1 : 0, left ? 1 : 0, left ? -1 : 0}, ctr,
                      {kPedSteps, kMoved, kEvacuated, kLive});
}

// ---- caller-order output ---------------------------------------------------------------

template <typename T>
__global__ void k_scatter(const T *__restrict__ src, const int32_t *__restrict__ ext,
                          T *__restrict__ dst, int n, T mask)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (size_t)n) dst[ext[i]] = src[i] & mask;
}

// Rows of a pitched field array into dense rows: dst[y * W + x] = src[y * fp + x].
template <typename T>
__global__ void k_copy_rows(const T *__restrict__ src, int fp, T *__restrict__ dst, int W, int H)
{
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (size_t)W * H) return;
    const size_t y = c / (size_t)W, x = c - y * (size_t)W;
    dst[c] = src[y * (size_t)fp + x];
}

// ---- batched counter read-out --------------------------------------------------------
//
// Workgroup j sums the slot copies of every running total of scene j into
// out[j * 16 + (0: step, 1 + id: total id)]: the slot copies are summed,
// except those of the running maximum kMaxClaim.

__global__ __launch_bounds__(64) void k_sum_counters(const SceneView *__restrict__ views,
                                                     unsigned long long *__restrict__ out)
{
    const gptr<const unsigned long long> ctr =
        to_global((const unsigned long long *)views[blockIdx.x].ctr);
    const int lane = (int)threadIdx.x;
    unsigned long long mine = 0;
    for (int id = 0; id < kNumCounters; ++id) {
        unsigned long long v = ctr[ctr_index(id, lane)];
        for (int d = 32; d >= 1; d >>= 1) {
            const unsigned long long o = __shfl_xor(v, d);
            v = id == kMaxClaim ? max(v, o) : v + o;
        }
        if (lane == 1 + id) mine = v;
    }
    if (lane == 0) mine = ctr[0];
    if (lane < 16) out[(size_t)blockIdx.x * 16 + lane] = mine;
}

// Plain launch, or a launch whose dispatch records `ev` (kernel timing).
template <typename K, typename... A>
hipError_t launch(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                  const LaunchEvents *ev, A... args)
{
    if (ev && ev->start)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, ev->start, ev->stop, 0u,
                              args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
    return hipGetLastError();
}

// Workgroups for n elements of bs threads, at most `cap`: grid-stride kernels
// take the default cap; kernels with one thread per element pass kCoverAll
// (n < 2^31 elements fit it).
constexpr unsigned int kCoverAll = 1u << 30;
inline unsigned int blocks_for(size_t n, unsigned int bs, unsigned int cap = 65535u * 16u)
{
    size_t b = (n + bs - 1) / bs;
    if (b == 0) b = 1;
    return (unsigned int)(b > cap ? cap : b);
}

template <int TW, int HL>
hipError_t sup_launch(const SupCfg &c, const unsigned long long *bits, int wpr, const double *tab,
                      double *out, int W, int H, hipStream_t st)
{
    constexpr int TH = (64 / TW) * HL;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int n_tiles = tiles_x * tiles_y;
    const int want = (n_tiles + kSupThreads / 64 - 1) / (kSupThreads / 64);
    const int grid = want < c.grid ? want : c.grid;
    hipLaunchKernelGGL((k_superpose<TW, HL>), dim3(grid > 0 ? grid : 1), dim3(kSupThreads),
                       c.lds_bytes, st, bits, wpr, tab, c.ncols * c.stride, c.stride, c.padx,
                       c.pady, c.radius, out, W, H, tiles_x, n_tiles);
    return hipGetLastError();
}

}  // namespace

// ---- launch configuration -------------------------------------------------------------

SupCfg make_sup_cfg(int radius, int tw, int hl, size_t elem)
{
    SupCfg c;
    c.tw = tw;
    c.hl = hl;
    c.g = 64 / tw;
    c.th = c.g * hl;
    c.radius = radius;
    c.padx = radius + tw - 1;
    c.pady = radius + c.th - 1;
    c.ncols = 2 * c.padx + 1;
    c.nrows = 2 * c.pady + 1;
    // stride = G * odd: lane l = col*G + rg reads word col*stride + rg (+ const),
    // and col*stride mod 64 = G * (col*odd mod TW) is a permutation of the
    // multiples of G, so the 64 lanes of a read hit 64 distinct banks (and the
    // two 32-lane halves 32 distinct banks each).
    int s = c.nrows;
    while (s % c.g != 0 || ((s / c.g) & 1) == 0) ++s;
    c.stride = s;
    c.elem = elem;
    c.lds_bytes = (size_t)c.ncols * c.stride * elem;
    return c;
}

// ---- launchers ----------------------------------------------------------------------

hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_field_sect(const SectView &v, int grid, bool update, bool image,
                             hipStream_t st, const LaunchEvents *ev)
{
    if (v.R > kSectMaxR) return hipErrorInvalidValue;
    const int tiles = ((v.W + 63) / 64) * ((v.H + kSectWaves * kSectHL - 1) / (kSectWaves * kSectHL));
    const dim3 g((unsigned)std::max(1, std::min(grid, tiles))), b(kSectWaves * 64);
    const bool sectacc = image && v.K != 8;
    if (update) {
        if (!image) return launch(k_field_sect<true, false, false>, g, b, 0, st, ev, v, tiles);
        if (sectacc) return launch(k_field_sect<true, true, true>, g, b, 0, st, ev, v, tiles);
        return launch(k_field_sect<true, true, false>, g, b, 0, st, ev, v, tiles);
    }
    if (!image) return launch(k_field_sect<false, false, false>, g, b, 0, st, ev, v, tiles);
    if (sectacc) return launch(k_field_sect<false, true, true>, g, b, 0, st, ev, v, tiles);
    return launch(k_field_sect<false, true, false>, g, b, 0, st, ev, v, tiles);
}

hipError_t launch_occ_mark(const int32_t *pos, int n, unsigned long long *occ, int wpr, int W,
                           int nsu, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_occ_mark, dim3(blocks_for((size_t)n, 256, kCoverAll)), dim3(256), 0, st,
                       pos, n, occ, wpr, W, nsu);
    return hipGetLastError();
}

hipError_t launch_stamp_fill(void *tab, int elem, double q, int n, int ncols, int stride,
                             int padx, int pady, int R, const float *oct, hipStream_t st)
{
    const int total = (R + 1) * (R + 2) / 2;
    for (int first = 0; first < total; first += kOctChunk) {
        OctChunk c;
        c.first = first;
        c.count = std::min(kOctChunk, total - first);
        for (int i = 0; i < c.count; ++i) c.v[i] = oct[first + i];
        for (int i = c.count; i < kOctChunk; ++i) c.v[i] = 0.f;
        hipLaunchKernelGGL(k_stamp_fill, dim3(blocks_for((size_t)n, 256, 1024)), dim3(256), 0, st,
                           tab, elem, q, n, ncols, stride, padx, pady, R, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_mask_to_bits(const uint8_t *mask, unsigned long long *bits, int W, int H, int wpr,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_mask_to_bits, dim3(blocks_for((size_t)wpr * H, 256, 8192)), dim3(256), 0,
                       st, mask, bits, W, H, wpr);
    return hipGetLastError();
}

hipError_t launch_bfs_seed(const uint8_t *exitm, int32_t *D, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_bfs_seed, dim3(blocks_for(n, 256, kCoverAll)), dim3(256), 0, st, exitm,
                       D, n);
    return hipGetLastError();
}

int bfs_levels_per_launch() { return kBfsLevels; }
int bfs_ring() { return kBfsRing; }

hipError_t launch_bfs_block(const unsigned long long *obits, unsigned long long *const vis[2],
                            unsigned long long *const fr[2], int32_t *D, int W, int H, int wpr,
                            int j, unsigned int *active, hipStream_t st)
{
    const dim3 grid((unsigned)((wpr + kBfsTileWords - 1) / kBfsTileWords),
                    (unsigned)((H + kBfsTileRows - 1) / kBfsTileRows));
    hipLaunchKernelGGL(k_bfs_block, grid, dim3(kBfsThreads), 0, st, obits, vis[j & 1], fr[j & 1],
                       vis[(j + 1) & 1], fr[(j + 1) & 1], D, W, H, wpr, j, active);
    return hipGetLastError();
}

hipError_t launch_count_unreachable(const uint8_t *obst, const int32_t *D, int n,
                                    unsigned long long *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_unreachable, dim3(blocks_for(n, 256, kCoverAll)), dim3(256), 0, st,
                       obst, D, n, out);
    return hipGetLastError();
}

hipError_t set_superpose_lds_limit(size_t f64_bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_superpose<8, 1>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)f64_bytes);
}

// ---- source-list gather: configuration and launch ------------------------------------

namespace {

// Most lanes of one LDS read of a source's stamp column that share a bank:
// lane l (column l % tw, row group l / tw) reads the entry at col*stride + rg
// (+ a uniform offset).  Measured on gfx950 with a probe: ds_read2_b64 (8-byte
// entries) serves a wave in passes of 16 consecutive lanes, conflict-free when
// their entry indices are distinct modulo 16; ds_read2_b32 (4-byte entries) in
// passes of 32 lanes, conflict-free when distinct modulo 32.  An n-way
// conflict costs up to n times a conflict-free pass (16-column tiles of
// doubles: an odd stride runs at the rate of a broadcast read, a stride of
// 2 mod 4 takes 1.6-1.75x as long, 4 mod 8 about 2.8x, 8 mod 16 about 5.6x).
// 16-byte loads (ds_read_b128; lane l reads the four integers from
// col*stride + 4*rg, stride a multiple of 4) run in passes of 32 lanes,
// conflict-free when their 16-byte units are distinct modulo 32 (probe: a
// conflict-free pass moves about 280 bytes per clock, against about 130 for
// the paired 4-byte loads; a 2-way conflict about 170).
int bank_degree(int tw, int stride, int elem, int vec = 2, int hl = 4)
{
    if (vec == 4) {
        // lane l's first load: integer col*stride + hl*rg, 16-byte unit
        // col*stride/4 + (hl/4)*rg (later loads of an hl = 8 lane: the next unit)
        int worst = 0;
        for (int p = 0; p < 64; p += 32) {
            int hits[32] = {0};
            for (int l = p; l < p + 32; ++l) {
                const int col = l % tw, rg = l / tw;
                ++hits[(col * (stride / 4) + (hl / 4) * rg) % 32];
            }
            for (int b = 0; b < 32; ++b) worst = hits[b] > worst ? hits[b] : worst;
        }
        return worst;
    }
    const int lanes = elem == 8 ? 16 : 32;
    int worst = 0;
    for (int p = 0; p < 64; p += lanes) {
        int hits[32] = {0};
        for (int l = p; l < p + lanes; ++l) {
            const int col = l % tw, rg = l / tw;
            ++hits[(col * stride + rg) % lanes];
        }
        for (int b = 0; b < lanes; ++b) worst = hits[b] > worst ? hits[b] : worst;
    }
    return worst;
}

}  // namespace

ListCfg make_list_cfg(int radius, int tw, int hl, int nw, int list_cap, int elem, int vec)
{
    ListCfg c;
    c.elem = elem;
    c.vec = vec;
    c.tw = tw;
    c.hl = hl;
    c.nw = nw;
    c.g = 64 / tw;
    c.th = c.g * hl;
    c.wt = nw * c.th;
    c.radius = radius;
    c.padx = radius + tw;
    c.pady = radius + c.th - 1;
    c.ncols = 2 * c.padx + 1;
    c.nrows = 2 * c.pady + 1;
    // A column holds the band |dy| <= R at rows pady - R .. pady + R; a read
    // reaches up to TH - 1 rows past the band on either side.  With stride >=
    // 2R + TH those reads land on zero rows of the same column or of the
    // neighbouring column (the next column's band starts TH - 1 rows into
    // it), so the columns need not hold all nrows rows; one zero column more
    // at the end takes the last column's overrun.
    const int smin = 2 * radius + c.th;
    int best = -1, best_deg = 1 << 30;
    for (int s = smin; s < smin + 64; ++s) {
        if (vec == 4 && s % 4 != 0) continue;  // lane rows 16-byte aligned in every column
        const int d = bank_degree(tw, s, elem, vec, hl);
        if (d < best_deg) {
            best_deg = d;
            best = s;
        }
        if (d == 1) break;
    }
    c.stride = best;
    // loaded as 16-byte vectors: 2 doubles or 4 integers each
    const int per_vec = 16 / elem;
    c.tab_elems = ((c.ncols + 1) * c.stride + per_vec - 1) / per_vec * per_vec;
    c.lds_tab = vec == 4 ? 4 * c.tab_elems + 4 : c.tab_elems;
    c.max_row = tw + 2 * radius;
    c.list_cap = list_cap;
    c.halo_rows = c.wt + 2 * radius;
    c.lds_bytes = (size_t)c.lds_tab * elem + (size_t)list_cap * 4 +
                  (size_t)(c.halo_rows + 1) * 4;
    return c;
}

ListCfg pick_list_cfg(int radius, size_t max_lds, int elem)
{
    // Integer stamps: 16-byte loads (four stamp copies) with two workgroups of
    // 8 or 4 waves per CU when LDS allows, else one workgroup of 16 waves
    // (large radii).  Otherwise, and for FP64 stamps: 16-column strips, two
    // entries per paired LDS read, two workgroups per CU preferred, smaller
    // lists and workgroups if LDS is short.
    if (elem == 4) {
        const int v4[][3] = {{16, 4, 8}, {16, 4, 4}, {16, 4, 16}};
        for (int i = 0; i < 3; ++i) {
            const int *sh = v4[i];
            for (int cap = 4096; cap >= 1024; cap /= 2) {
                ListCfg t = make_list_cfg(radius, sh[0], sh[1], sh[2], cap, elem, 4);
                if (cap < 2 * t.max_row || t.halo_rows > 64 * sh[2]) break;
                if (t.lds_bytes <= (sh[2] == 16 ? max_lds : max_lds / 2)) return t;
            }
        }
    }
    const int shapes[][3] = {{16, 2, 8}, {16, 2, 4}};
    ListCfg best;
    for (int i = 0; i < 2; ++i) {
        const int *sh = shapes[i];
        for (int cap = 4096; cap >= 512; cap /= 2) {
            ListCfg t = make_list_cfg(radius, sh[0], sh[1], sh[2], cap, elem);
            if (cap < 2 * t.max_row || t.halo_rows > 64 * sh[2]) break;
            if (t.lds_bytes <= max_lds / 2) return t;
            if (t.lds_bytes <= max_lds && best.lds_bytes == 0) best = t;
        }
    }
    return best;
}

void set_view_layout(SceneView &v, const ListCfg &c, const double *tab, const int32_t *tabi,
                     double q, int int_rounds)
{
    v.int_rounds = int_rounds;
    v.tiles_x = (v.W + c.tw - 1) / c.tw;
    v.n_strips = v.tiles_x * ((v.H + c.wt - 1) / c.wt);
    v.stride = c.stride;
    v.padx = c.padx;
    v.pady = c.pady;
    v.max_row = c.max_row;
    v.tab_elems = c.tab_elems;
    v.tab = tab;
    v.tabi = tabi;
    v.q = q;
}

FieldLaunch field_launch_for(const ListCfg &c)
{
    FieldLaunch f;
    f.tw = c.tw;
    f.hl = c.hl;
    f.nw = c.nw;
    f.list_cap = c.list_cap;
    f.tab_max = c.lds_tab;
    f.halo_max = c.halo_rows;
    f.grid = c.grid;
    f.elem = c.elem;
    f.vec = c.vec;
    f.lds_bytes = field_lds_bytes(f);
    return f;
}

size_t field_lds_bytes(const FieldLaunch &f)
{
    return (size_t)f.tab_max * f.elem + (size_t)f.list_cap * 4 + (size_t)(f.halo_max + 1) * 4;
}

// Compiled shapes (strip width TW, rows per lane HL, waves per workgroup NW);
// the 16-byte-load shapes (VEC = 4) are compiled for integer stamps only.
#define SF_LIST_SHAPES(X)                                                                     \
    X(16, 2, 4) X(16, 2, 8) X(16, 4, 4) X(16, 4, 8) X(32, 2, 4) X(32, 2, 8) X(32, 4, 4)         \
    X(8, 2, 4) X(8, 4, 4)
#define SF_V4_SHAPES(X) X(16, 4, 4) X(16, 4, 8) X(32, 4, 4) X(8, 4, 4) X(32, 8, 4) X(16, 8, 4)
// 16 waves: for stamps large enough that one workgroup fills a CU's LDS
#define SF_V4_WIDE(X) X(16, 4, 16)

bool list_shape_compiled(int tw, int hl, int nw, int vec, int elem)
{
#define SF_KNOWN(a, b, n) \
    if (tw == a && hl == b && nw == n) return true;
    if (vec == 2) {
        SF_LIST_SHAPES(SF_KNOWN)
    } else if (vec == 4 && elem == 4) {
        SF_V4_SHAPES(SF_KNOWN)
        SF_V4_WIDE(SF_KNOWN)
    }
#undef SF_KNOWN
    return false;
}

hipError_t set_field_lds_limit(size_t bytes)
{
    hipError_t e = hipSuccess;
#define SF_SET1(...)                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_field<__VA_ARGS__>),             \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);          \
    if (e != hipSuccess) return e;
#define SF_SET(a, b, n)                                                                          \
    SF_SET1(a, b, n, false, false, false) SF_SET1(a, b, n, true, false, false)                 \
    SF_SET1(a, b, n, false, true, false) SF_SET1(a, b, n, false, false, true)                  \
    SF_SET1(a, b, n, true, false, true) SF_SET1(a, b, n, false, true, true)
#define SF_SET4(a, b, n)                                                                         \
    SF_SET1(a, b, n, false, false, true, 4) SF_SET1(a, b, n, true, false, true, 4)             \
    SF_SET1(a, b, n, false, true, true, 4)
    SF_LIST_SHAPES(SF_SET)
    SF_V4_SHAPES(SF_SET4)
    SF_V4_WIDE(SF_SET4)
#undef SF_SET4
#undef SF_SET
#undef SF_SET1
    return hipSuccess;
}

hipError_t launch_field(const FieldLaunch &f, const SceneView *views, const int32_t *items,
                        int n_items, unsigned int *queue, hipStream_t st, const LaunchEvents *ev)
{
    const int grid = std::max(1, std::min(f.grid, n_items));
    const int4 *it = reinterpret_cast<const int4 *>(items);
    const SceneView none = {};
#define SF_DISPATCH4(a, b, n)                                                                     \
    if (f.tw == a && f.hl == b && f.nw == n)                                                    \
        return launch(k_field<a, b, n, true, false, true, 4>, dim3(grid), dim3(n * 64),          \
                      f.lds_bytes, st, ev, none, views, it, n_items, 0, f.tab_max, f.list_cap,    \
                      queue);
    if (f.vec == 4) {
        if (f.elem != 4) return hipErrorInvalidValue;
        SF_V4_SHAPES(SF_DISPATCH4)
        SF_V4_WIDE(SF_DISPATCH4)
        return hipErrorInvalidValue;
    }
#undef SF_DISPATCH4
#define SF_DISPATCH(a, b, n)                                                                      \
    if (f.tw == a && f.hl == b && f.nw == n)                                                    \
        return f.elem == 4                                                                      \
                   ? launch(k_field<a, b, n, true, false, true>, dim3(grid), dim3(n * 64),      \
                            f.lds_bytes, st, ev, none, views, it, n_items, 0, f.tab_max,        \
                            f.list_cap, queue)                                                  \
                   : launch(k_field<a, b, n, true, false, false>, dim3(grid), dim3(n * 64),     \
                            f.lds_bytes, st, ev, none, views, it, n_items, 0, f.tab_max,        \
                            f.list_cap, queue);
    SF_LIST_SHAPES(SF_DISPATCH)
#undef SF_DISPATCH
    return hipErrorInvalidValue;
}

int field_resident_blocks(int tw, int hl, int nw, size_t lds_bytes, bool multi, int elem, int vec)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    const void *fn = nullptr;
    if (vec == 4) {
        if (elem != 4) return 0;
#define SF_OCC4(a, b, w)                                                                          \
    if (tw == a && hl == b && nw == w) {                                                         \
        fn = multi ? reinterpret_cast<const void *>(&k_field<a, b, w, true, false, true, 4>)      \
                   : reinterpret_cast<const void *>(&k_field<a, b, w, false, false, true, 4>);    \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, w * 64, lds_bytes);             \
    }
        SF_V4_SHAPES(SF_OCC4)
        SF_V4_WIDE(SF_OCC4)
#undef SF_OCC4
        return e == hipSuccess ? n : 0;
    }
#define SF_OCC(a, b, w)                                                                           \
    if (tw == a && hl == b && nw == w) {                                                         \
        if (elem == 4)                                                                           \
            fn = multi ? reinterpret_cast<const void *>(&k_field<a, b, w, true, false, true>)     \
                       : reinterpret_cast<const void *>(&k_field<a, b, w, false, false, true>);   \
        else                                                                                     \
            fn = multi ? reinterpret_cast<const void *>(&k_field<a, b, w, true, false, false>)    \
                       : reinterpret_cast<const void *>(&k_field<a, b, w, false, false, false>);  \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, w * 64, lds_bytes);             \
    }
    SF_LIST_SHAPES(SF_OCC)
#undef SF_OCC
    return e == hipSuccess ? n : 0;
}

hipError_t launch_field_dense(const SceneView &view, int grid, hipStream_t st,
                              const LaunchEvents *ev)
{
    const int tiles = ((view.W + 63) / 64) * ((view.H + kDenseWaves * kDenseHL - 1) /
                                                (kDenseWaves * kDenseHL));
    const dim3 g((unsigned)std::max(1, std::min(grid, tiles))), b(kDenseWaves * 64);
    switch (view.R) {
    case 1: return launch(k_field_dense<1>, g, b, 0, st, ev, view, tiles);
    case 2: return launch(k_field_dense<2>, g, b, 0, st, ev, view, tiles);
    case 3: return launch(k_field_dense<3>, g, b, 0, st, ev, view, tiles);
    case 4: return launch(k_field_dense<4>, g, b, 0, st, ev, view, tiles);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_field_one(const FieldLaunch &f, const SceneView &view, int per,
                            hipStream_t st, const LaunchEvents *ev)
{
    const int n_items = std::max(1, (view.n_strips + per - 1) / per);
    const int grid = std::max(1, std::min(f.grid, n_items));
#define SF_DISPATCH4(a, b, n)                                                                     \
    if (f.tw == a && f.hl == b && f.nw == n)                                                    \
        return launch(k_field<a, b, n, false, false, true, 4>, dim3(grid), dim3(n * 64),         \
                      f.lds_bytes, st, ev, view, (const SceneView *)nullptr,                    \
                      (const int4 *)nullptr, n_items, per, f.tab_max, f.list_cap,       \
                      (unsigned int *)nullptr);
    if (f.vec == 4) {
        if (f.elem != 4) return hipErrorInvalidValue;
        SF_V4_SHAPES(SF_DISPATCH4)
        SF_V4_WIDE(SF_DISPATCH4)
        return hipErrorInvalidValue;
    }
#undef SF_DISPATCH4
#define SF_DISPATCH(a, b, n)                                                                      \
    if (f.tw == a && f.hl == b && f.nw == n)                                                    \
        return f.elem == 4                                                                      \
                   ? launch(k_field<a, b, n, false, false, true>, dim3(grid), dim3(n * 64),     \
                            f.lds_bytes, st, ev, view, (const SceneView *)nullptr,              \
                            (const int4 *)nullptr, n_items, per, f.tab_max, f.list_cap,       \
                      (unsigned int *)nullptr)         \
                   : launch(k_field<a, b, n, false, false, false>, dim3(grid), dim3(n * 64),    \
                            f.lds_bytes, st, ev, view, (const SceneView *)nullptr,              \
                            (const int4 *)nullptr, n_items, per, f.tab_max, f.list_cap,       \
                      (unsigned int *)nullptr);
    SF_LIST_SHAPES(SF_DISPATCH)
#undef SF_DISPATCH
    return hipErrorInvalidValue;
}

hipError_t launch_field_update(const FieldLaunch &f, const SceneView &view, int per,
                               hipStream_t st, const LaunchEvents *ev)
{
    const int n_items = std::max(1, (view.n_strips + per - 1) / per);
    const int grid = std::max(1, std::min(f.grid, n_items));
#define SF_DISPATCH4(a, b, n)                                                                     \
    if (f.tw == a && f.hl == b && f.nw == n)                                                    \
        return launch(k_field<a, b, n, false, true, true, 4>, dim3(grid), dim3(n * 64),          \
                      f.lds_bytes, st, ev, view, (const SceneView *)nullptr,                    \
                      (const int4 *)nullptr, n_items, per, f.tab_max, f.list_cap,       \
                      (unsigned int *)nullptr);
    if (f.vec == 4) {
        if (f.elem != 4) return hipErrorInvalidValue;
        SF_V4_SHAPES(SF_DISPATCH4)
        SF_V4_WIDE(SF_DISPATCH4)
        return hipErrorInvalidValue;
    }
#undef SF_DISPATCH4
#define SF_DISPATCH(a, b, n)                                                                      \
    if (f.tw == a && f.hl == b && f.nw == n)                                                    \
        return f.elem == 4                                                                      \
                   ? launch(k_field<a, b, n, false, true, true>, dim3(grid), dim3(n * 64),      \
                            f.lds_bytes, st, ev, view, (const SceneView *)nullptr,              \
                            (const int4 *)nullptr, n_items, per, f.tab_max, f.list_cap,       \
                      (unsigned int *)nullptr)         \
                   : launch(k_field<a, b, n, false, true, false>, dim3(grid), dim3(n * 64),     \
                            f.lds_bytes, st, ev, view, (const SceneView *)nullptr,              \
                            (const int4 *)nullptr, n_items, per, f.tab_max, f.list_cap,       \
                      (unsigned int *)nullptr);
    SF_LIST_SHAPES(SF_DISPATCH)
#undef SF_DISPATCH
    return hipErrorInvalidValue;
}

hipError_t launch_superpose_f64(const SupCfg &c, const unsigned long long *bits, int wpr,
                                const double *tab, double *out, int W, int H, hipStream_t st)
{
    if (c.tw == 8 && c.hl == 1) return sup_launch<8, 1>(c, bits, wpr, tab, out, W, H, st);
    return hipErrorInvalidValue;
}

hipError_t launch_static_S(const int32_t *D, const double *O, const uint8_t *obst, double w_dest,
                           double *S, int W, int H, int fp, hipStream_t st)
{
    const int n = W * H;
    hipLaunchKernelGGL(k_static_S, dim3(blocks_for(n, 256, kCoverAll)), dim3(256), 0, st, D, O,
                       obst, w_dest, S, W, H, fp);
    return hipGetLastError();
}

hipError_t launch_occ_init(const int32_t *pos, int N, unsigned long long *occ, int wpr, int W,
                           unsigned long long *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_occ_init, dim3(blocks_for(N, 256, kCoverAll)), dim3(256), 0, st, pos, N,
                       occ, wpr, W, ctr);
    return hipGetLastError();
}

int decide_blocks(int N) { return decide_block_count(N); }

int commit_blocks(int N)
{
    return (int)blocks_for((size_t)N, commit_threads<true>(), 1u << 30);
}

hipError_t launch_decide_claim(const SceneView *views, const int32_t *block_scene, int n_blocks,
                               hipStream_t st, const LaunchEvents *ev)
{
    const SceneView none = {};
    return launch(k_decide_claim<true>, dim3(n_blocks), dim3(kDecideThreads), 0, st, ev, none,
                  views, block_scene);
}

hipError_t launch_decide_one(const SceneView &view, hipStream_t st, const LaunchEvents *ev)
{
    return launch(k_decide_claim<false>, dim3(decide_blocks(view.N)), dim3(kDecideThreads), 0, st,
                  ev, view, (const SceneView *)nullptr, (const int32_t *)nullptr);
}

hipError_t launch_clear_claims(ClaimRec *c, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_claims, dim3(blocks_for(n, 256, kCoverAll)), dim3(256), 0, st, c, n);
    return hipGetLastError();
}

hipError_t launch_scatter_i32(const int32_t *src, const int32_t *ext, int32_t *dst, int n,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter<int32_t>, dim3(blocks_for((size_t)n, 256, kCoverAll)), dim3(256),
                       0, st, src, ext, dst, n, (int32_t)-1);
    return hipGetLastError();
}

hipError_t launch_scatter_u8(const uint8_t *src, const int32_t *ext, uint8_t *dst, int n,
                             uint8_t mask, hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter<uint8_t>, dim3(blocks_for((size_t)n, 256, kCoverAll)), dim3(256),
                       0, st, src, ext, dst, n, mask);
    return hipGetLastError();
}

hipError_t launch_copy_rows(const void *src, int fp, void *dst, int W, int H, int elem,
                            hipStream_t st)
{
    const size_t n = (size_t)W * H;
    if (n == 0) return hipSuccess;
    if (elem == 4)
        hipLaunchKernelGGL(k_copy_rows<uint32_t>, dim3(blocks_for(n, 256, kCoverAll)), dim3(256),
                           0, st, static_cast<const uint32_t *>(src), fp,
                           static_cast<uint32_t *>(dst), W, H);
    else if (elem == 8)
        hipLaunchKernelGGL(k_copy_rows<unsigned long long>, dim3(blocks_for(n, 256, kCoverAll)),
                           dim3(256), 0, st, static_cast<const unsigned long long *>(src), fp,
                           static_cast<unsigned long long *>(dst), W, H);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_sum_counters(const SceneView *views, int n_scenes, unsigned long long *out,
                               hipStream_t st)
{
    static_assert(kSlots == 64 && kNumCounters <= 15, "one lane per slot, 16 words per scene");
    hipLaunchKernelGGL(k_sum_counters, dim3(n_scenes), dim3(64), 0, st, views, out);
    return hipGetLastError();
}

hipError_t launch_commit(const SceneView *views, const int32_t *block_scene, int n_blocks,
                         hipStream_t st, const LaunchEvents *ev)
{
    const SceneView none = {};
    return launch(k_commit<true>, dim3(n_blocks), dim3(commit_threads<true>()), 0, st, ev, none,
                  views, block_scene);
}

hipError_t launch_body_init(const SceneView &view, hipStream_t st)
{
    hipLaunchKernelGGL(k_body_init, dim3(blocks_for((size_t)view.N, 256, kCoverAll)), dim3(256), 0,
                       st, view);
    return hipGetLastError();
}

hipError_t launch_decide_body(const SceneView &view, hipStream_t st, const LaunchEvents *ev)
{
    return launch(k_decide_body, dim3(decide_blocks(view.N)), dim3(kDecideThreads), 0, st, ev,
                  view);
}

hipError_t launch_commit_body(const SceneView &view, hipStream_t st, const LaunchEvents *ev)
{
    return launch(k_commit_body, dim3(blocks_for((size_t)view.N, 256, 1u << 30)), dim3(256), 0,
                  st, ev, view);
}

hipError_t launch_commit_one(const SceneView &view, hipStream_t st, const LaunchEvents *ev)
{
    constexpr int nt = commit_threads<false>();
    return launch(k_commit<false>, dim3(blocks_for((size_t)view.N, nt, 1u << 30)), dim3(nt), 0, st,
                  ev, view, (const SceneView *)nullptr, (const int32_t *)nullptr);
}

}  // namespace sf
