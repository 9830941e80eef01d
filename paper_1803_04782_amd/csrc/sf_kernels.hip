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

#include <cmath>
#include <cstdint>

#include "sf_internal.h"

namespace sf {

namespace {

constexpr int kDirX[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
constexpr int kDirY[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};

constexpr uint8_t kMover = 1u, kWon = 2u, kTied = 4u;

// ---- small helpers ------------------------------------------------------------

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Sum of `v` over the block, added by one thread to copy (block % kSlots) of
// running total `id` (skipped when 0).  Every thread of the block must call
// it; it synchronises the block.
__device__ __forceinline__ void block_sum_add(unsigned int v, unsigned long long *ctr, int id)
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
        if (s) atomicAdd(&ctr[ctr_index(id, blockIdx.x % kSlots)], s);
    }
    __syncthreads();
}

// Same for a signed delta (two's-complement add).
__device__ __forceinline__ void block_delta_add(int v, unsigned long long *ctr, int id)
{
    __shared__ int part[16];
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) part[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long s = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
        if (s) atomicAdd(&ctr[ctr_index(id, blockIdx.x % kSlots)], (unsigned long long)s);
    }
    __syncthreads();
}

// Wave-aggregated append: lanes with `pred` get consecutive slots of a list
// whose length is *cnt; one atomic per wave.
__device__ __forceinline__ unsigned int wave_append(bool pred, unsigned int *cnt)
{
    const unsigned long long b = __ballot(pred);
    if (b == 0) return 0;
    unsigned int base = 0;
    const int leader = __ffsll((long long)b) - 1;
    if ((int)lane_id() == leader) base = atomicAdd(cnt, (unsigned int)__popcll(b));
    base = __shfl(base, leader);
    const unsigned long long below = b & ((1ull << lane_id()) - 1ull);
    return base + (unsigned int)__popcll(below);
}

// Pointer into LDS (address space 3): 32-bit byte addresses, ds_* instructions.
template <typename T>
using lds_ptr = const __attribute__((address_space(3))) T *;

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

// ---- field law table ----------------------------------------------------------

// Column-major, zero-padded stamp: entry (dx, dy) at (dx+padx)*stride +
// (dy+pady) holds k*|d|^alpha inside the square window, 0 elsewhere and at
// d = 0.  Evaluated in FP64 and rounded once to T.
template <typename T>
__global__ void k_phi_table(T *tab, int ncols, int nrows, int stride, int padx, int pady, int R,
                            double k, double alpha)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncols * stride) return;
    const int ci = i / stride, ri = i - ci * stride;
    const int dx = ci - padx, dy = ri - pady;
    double v = 0.0;
    if (ri < nrows && abs(dx) <= R && abs(dy) <= R && (dx != 0 || dy != 0))
        v = k * pow(sqrt((double)dx * dx + (double)dy * dy), alpha);
    tab[i] = (T)v;
}

// ---- destination field: multi-source BFS --------------------------------------

__global__ void k_bfs_init(const uint8_t *__restrict__ obst, const uint8_t *__restrict__ exitm,
                           int32_t *__restrict__ D, int32_t *__restrict__ frontier,
                           unsigned int *cnt, int n)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    bool src = false;
    if (c < n) {
        src = exitm[c] && !obst[c];
        D[c] = src ? 0 : -1;
    }
    const unsigned int slot = wave_append(src, &cnt[0]);
    if (src) frontier[slot] = c;
}

// Expansion of BFS level L: frontier of level L (count cnt[L%3]) -> level L+1
// (count cnt[(L+1)%3]); cnt[(L+2)%3] is cleared for the next launch.
__global__ void k_bfs_expand(const uint8_t *__restrict__ obst, int32_t *D,
                             const int32_t *__restrict__ fin, int32_t *__restrict__ fout,
                             unsigned int *cnt, int W, int H, int L)
{
    const unsigned int n_in = cnt[L % 3];
    const unsigned int nthreads = gridDim.x * blockDim.x;
    const unsigned int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) cnt[(L + 2) % 3] = 0u;
    // every lane of a wave runs the same number of iterations (wave_append
    // needs the whole wave)
    const unsigned int rounds = (n_in + nthreads - 1) / nthreads;
    for (unsigned int r = 0; r < rounds; ++r) {
        const unsigned int i = r * nthreads + tid;
        const bool act = i < n_in;
        int x = 0, y = 0;
        if (act) {
            const int c = fin[i];
            x = c % W;
            y = c / W;
        }
#pragma unroll
        for (int d = 1; d <= 8; ++d) {
            const int nx = x + kDirX[d], ny = y + kDirY[d];
            bool found = false;
            int nc = 0;
            if (act && nx >= 0 && ny >= 0 && nx < W && ny < H) {
                nc = ny * W + nx;
                if (!obst[nc] && D[nc] < 0) found = atomicCAS(&D[nc], -1, L + 1) == -1;
            }
            const unsigned int slot = wave_append(found, &cnt[(L + 1) % 3]);
            if (found) fout[slot] = nc;
        }
    }
}

__global__ void k_count_unreachable(const uint8_t *__restrict__ obst, const int32_t *__restrict__ D,
                                    int n, unsigned long long *ctr)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const bool bad = c < n && !obst[c] && D[c] < 0;
    block_sum_add(bad ? 1u : 0u, ctr, kScratch);
}

__global__ void k_static_S(const int32_t *__restrict__ D, const double *__restrict__ O,
                           const uint8_t *__restrict__ obst, double w_dest, float *__restrict__ S,
                           int n)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    S[c] = obst[c] ? INFINITY : (float)(w_dest * (double)D[c] + O[c]);
}

// ---- field superposition --------------------------------------------------------

// Persistent kernel: each wave takes TW x TH output tiles.  For every live
// source in the tile's R-halo (bitmap words scanned in row-major order; the
// source coordinates are wave-uniform) each lane adds HL table entries, one
// per owned row, at immediate offsets G*r from a single per-source address.
constexpr int kSupThreads = 256;

template <typename T, int TW, int HL, bool ADD_S>
__global__ __launch_bounds__(kSupThreads) void k_superpose(
    const unsigned long long *__restrict__ bits, int wpr, const T *__restrict__ tab_g,
    int tab_elems, int stride, int padx, int pady, int R, const float *__restrict__ S,
    T *__restrict__ outT, float *__restrict__ outP, int W, int H, int tiles_x, int n_tiles)
{
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
            if (x < W && y < H) {
                const size_t c = (size_t)y * W + x;
                if constexpr (ADD_S)
                    outP[c] = S[c] + (float)acc[r];
                else
                    outT[c] = acc[r];
            }
        }
    }
}

// ---- per-tick field: source-list gather ---------------------------------------------
//
// One workgroup per TW-column strip of NW*TH rows (persistent over strips).
//  1. thread t loads the bitmap words of halo row ya + t and counts its sources;
//  2. a block-wide exclusive scan turns the counts into list offsets, so the
//     list holds the strip's halo sources in global row-major order;
//  3. each thread writes its row's entries: an entry is the byte offset that
//     turns a lane's base address into the address of table entry
//     (lane su - source) in the aligned copy for the source's row;
//  4. each wave walks the contiguous part of the list that lies within R rows
//     of its own rows: per source one address add, HL/VEC aligned LDS vector
//     loads and HL adds per lane.
// A halo with more than list_cap - max_row sources is processed in several
// passes over consecutive row ranges, which keeps the row-major order.

template <int VEC>
struct VecOf;
template <>
struct VecOf<2> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct VecOf<4> {
    typedef float type __attribute__((ext_vector_type(4)));
};

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

// acc[q] += table vector at LDS byte address a + q*sizeof(vec)
template <int NQ, typename V>
__device__ __forceinline__ void gather_one(V *acc, int a)
{
    typedef const __attribute__((address_space(3))) V *ptr;
    const ptr s = reinterpret_cast<ptr>((uint32_t)a);
    V v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = s[q];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += v[q];
}

template <int TW, int HL, int VEC, int NW>
__global__ __launch_bounds__(NW * 64) void k_field_list(
    const unsigned long long *__restrict__ bits, int wpr, const float *__restrict__ tab_g,
    int copy_elems, int stride, int padx, int pady, int R, int list_cap, int max_row,
    const float *__restrict__ S, float *__restrict__ P, int W, int H, int tiles_x, int n_tiles)
{
    constexpr int G = 64 / TW, TH = G * HL, WT = NW * TH, NT = NW * 64, NQ = HL / VEC;
    typedef typename VecOf<VEC>::type vec_t;
    typedef const __attribute__((address_space(3))) vec_t *lds_vec;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int wave_tot[NW];
    float *tab = reinterpret_cast<float *>(lds_raw);
    const int tab_elems = VEC * copy_elems;  // a multiple of 4
    int *list = reinterpret_cast<int *>(tab + tab_elems);
    int *row_excl = list + list_cap;
    for (int i = threadIdx.x; i < tab_elems / 4; i += NT)
        reinterpret_cast<float4 *>(tab)[i] = reinterpret_cast<const float4 *>(tab_g)[i];
    __syncthreads();

    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane % TW, rg = lane / TW;
    const int tbase = (int)(uint32_t)(uintptr_t)((lds_ptr<float>)tab);
    const int cap = list_cap - max_row;

    // Strip geometry: halo rows [ya, ya + nr), halo bitmap words [wa, wa + nwd).
    struct Strip {
        int X0, Y0, ya, nr, xa, xb, wa, nwd;
    };
    auto strip = [&](int t) {
        Strip g;
        const int ty = t / tiles_x, tx = t - ty * tiles_x;
        g.X0 = tx * TW;
        g.Y0 = ty * WT;
        g.ya = max(g.Y0 - R, 0);
        g.nr = min(g.Y0 + WT - 1 + R, H - 1) - g.ya + 1;
        g.xa = max(g.X0 - R, 0);
        g.xb = min(g.X0 + TW - 1 + R, W - 1);
        g.wa = g.xa >> 6;
        g.nwd = (g.xb >> 6) - g.wa + 1;
        return g;
    };
    // bitmap words of this thread's halo row of strip t (issued early: the
    // loads stay in flight across the previous strip's work)
    unsigned long long n0 = 0, n1 = 0, n2 = 0;
    auto fetch_rows = [&](int t) {
        n0 = n1 = n2 = 0;
        if (t >= n_tiles) return;
        const Strip g = strip(t);
        if (tid < g.nr) {
            const unsigned long long *row = bits + (size_t)(g.ya + tid) * wpr + g.wa;
            n0 = row[0];
            if (g.nwd > 1) n1 = row[1];
            if (g.nwd > 2) n2 = row[2];
        }
    };
    fetch_rows((int)blockIdx.x);

    for (int t = (int)blockIdx.x; t < n_tiles; t += (int)gridDim.x) {
        const Strip g = strip(t);
        const int X0 = g.X0, Y0 = g.Y0, y0w = Y0 + wv * TH;
        const int ya = g.ya, nr = g.nr, xa = g.xa, xb = g.xb, wa = g.wa, nwd = g.nwd;
        const int yb = ya + nr - 1;
        const unsigned long long ma = ~0ull << (xa & 63), mb = ~0ull >> (63 - (xb & 63));

        // 1. this thread's halo row
        unsigned long long m0 = n0, m1 = n1, m2 = n2;
        m0 &= ma;
        if (nwd == 1) m0 &= mb;
        if (nwd == 2) m1 &= mb;
        if (nwd == 3) m2 &= mb;
        const int cnt = __popcll(m0) + __popcll(m1) + __popcll(m2);
        // keep the loads below after the use of the prefetched words, so that
        // the wait for those does not also wait for the new requests
        asm volatile("" ::"v"(cnt) : "memory");
        // S of this lane's su and the next strip's halo rows are requested now
        // and arrive while this strip is gathered
        const int x = X0 + col;
        float sv[HL];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                const int y = y0w + rg * HL + q * VEC + j;
                sv[q * VEC + j] = (x < W && y < H) ? S[(size_t)y * W + x] : 0.0f;
            }
        }
        fetch_rows(t + (int)gridDim.x);

        // 2. block exclusive scan of the row counts (ballots within a wave)
        int wtot;
        const int wexcl = wave_excl_small(cnt, wtot);
        if (lane == 0) wave_tot[wv] = wtot;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int v = wave_tot[w];
            before += w < wv ? v : 0;
            total += v;
        }
        const int excl = before + wexcl;
        if (tid < nr) row_excl[tid] = excl;
        if (tid == 0) row_excl[nr] = total;
        __syncthreads();

        // this wave's halo rows (relative to ya) and per-lane base address
        const int ra = max(y0w - R, ya) - ya;
        const int rb = min(y0w + TH - 1 + R, yb) - ya;
        const int lb = opaque_lane(tbase + ((X0 + col + padx) * stride + (y0w + rg * HL + pady)) * 4);
        vec_t acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = (vec_t)(0.0f);

        const int npass = (total + cap - 1) / cap;
        for (int k = 0; k < npass; ++k) {
            int start = 0, end = total;
            if (npass > 1) {
                start = row_excl[lower_bound_lds(row_excl, nr, k * cap)];
                if (k + 1 < npass) end = row_excl[lower_bound_lds(row_excl, nr, (k + 1) * cap)];
            }
            // 3. entries of the rows in this pass
            if (tid < nr && cnt > 0 && excl >= start && excl < end) {
                const int py = ya + tid;
                const int c = (py - pady) & (VEC - 1);
                const int rowterm = c * copy_elems * 4 - (py - c) * 4;
                int o = excl - start;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    unsigned long long mj = j == 0 ? m0 : (j == 1 ? m1 : m2);
                    const int xw = (wa + j) * 64;
                    while (mj) {
                        const int b = __builtin_ctzll(mj);
                        mj &= mj - 1ull;
                        list[o++] = rowterm - (xw + b) * stride * 4;
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
                for (; i < hi && (i & 3); ++i) gather_one<NQ>(acc, lb + list[i]);
                const int4 *list4 = reinterpret_cast<const int4 *>(list);
                // eight sources per round: both entry groups are read first, then
                // eight table reads are in flight before the adds
                for (; i + 8 <= hi; i += 8) {
                    const int4 ea = list4[i >> 2];
                    const int4 eb = list4[(i >> 2) + 1];
                    const int a[8] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
                    vec_t v[8][NQ];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const lds_vec sp = reinterpret_cast<lds_vec>((uint32_t)(lb + a[u]));
#pragma unroll
                        for (int q = 0; q < NQ; ++q) v[u][q] = sp[q];
                    }
                    // row-major source order per accumulator
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) acc[q] += v[u][q];
                    }
                }
                if (i + 4 <= hi) {
                    const int4 ea = list4[i >> 2];
                    const int a[4] = {ea.x, ea.y, ea.z, ea.w};
                    vec_t v[4][NQ];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const lds_vec sp = reinterpret_cast<lds_vec>((uint32_t)(lb + a[u]));
#pragma unroll
                        for (int q = 0; q < NQ; ++q) v[u][q] = sp[q];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) acc[q] += v[u][q];
                    }
                    i += 4;
                }
                for (; i < hi; ++i) gather_one<NQ>(acc, lb + list[i]);
            }
            __syncthreads();
        }

        // 5. P = S + Phi for this lane's su
        if (x < W) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    const int y = y0w + rg * HL + q * VEC + j;
                    if (y < H) P[(size_t)y * W + x] = sv[q * VEC + j] + acc[q][j];
                }
            }
        }
        __syncthreads();  // wave_tot and row_excl are rewritten by the next strip
    }
}

// ---- per-tick field, wave-private source lists ----------------------------------------
//
// Same table, entries and gather as k_field_list, but every wave lists the
// sources of its own TW x TH tile's halo, so waves never wait for each other:
// lane i holds halo rows i, 64 + i and 128 + i; the row counts are prefix-summed
// with ballots (no LDS traffic); entries go to a wave-private LDS list of `cap`
// entries (several passes when a dense halo overflows it).

template <int TW, int HL, int VEC, int NW>
__global__ __launch_bounds__(NW * 64) void k_field_wave(
    const unsigned long long *__restrict__ bits, int wpr, const float *__restrict__ tab_g,
    int copy_elems, int stride, int padx, int pady, int R, int cap, int max_row,
    const float *__restrict__ S, float *__restrict__ P, int W, int H, int tiles_x, int n_tiles)
{
    constexpr int G = 64 / TW, TH = G * HL, NQ = HL / VEC, NS = 3;
    typedef typename VecOf<VEC>::type vec_t;
    typedef const __attribute__((address_space(3))) vec_t *lds_vec;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float *tab = reinterpret_cast<float *>(lds_raw);
    const int tab_elems = VEC * copy_elems;  // a multiple of 4
    for (int i = threadIdx.x; i < tab_elems / 4; i += NW * 64)
        reinterpret_cast<float4 *>(tab)[i] = reinterpret_cast<const float4 *>(tab_g)[i];
    __syncthreads();

    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    int *list = reinterpret_cast<int *>(tab + tab_elems) + wv * cap;  // cap: a multiple of 4
    const int col = lane % TW, rg = lane / TW;
    const int tbase = (int)(uint32_t)(uintptr_t)((lds_ptr<float>)tab);
    const int capp = cap - max_row;
    const int t0 = __builtin_amdgcn_readfirstlane((int)blockIdx.x * NW + wv);
    const int tstep = __builtin_amdgcn_readfirstlane((int)gridDim.x * NW);

    struct Tile {
        int X0, Y0, ya, nr, xa, xb, wa, nwd;
    };
    auto tile = [&](int t) {
        Tile g;
        const int ty = t / tiles_x, tx = t - ty * tiles_x;
        g.X0 = tx * TW;
        g.Y0 = ty * TH;
        g.ya = max(g.Y0 - R, 0);
        g.nr = min(g.Y0 + TH - 1 + R, H - 1) - g.ya + 1;
        g.xa = max(g.X0 - R, 0);
        g.xb = min(g.X0 + TW - 1 + R, W - 1);
        g.wa = g.xa >> 6;
        g.nwd = (g.xb >> 6) - g.wa + 1;
        return g;
    };
    unsigned long long n[NS][3];
    auto fetch = [&](int t) {
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) n[sl][0] = n[sl][1] = n[sl][2] = 0;
        if (t >= n_tiles) return;
        const Tile g = tile(t);
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const int r = 64 * sl + lane;
            if (r < g.nr) {
                const unsigned long long *row = bits + (size_t)(g.ya + r) * wpr + g.wa;
                n[sl][0] = row[0];
                if (g.nwd > 1) n[sl][1] = row[1];
                if (g.nwd > 2) n[sl][2] = row[2];
            }
        }
    };
    fetch(t0);

    for (int t = t0; t < n_tiles; t += tstep) {
        const Tile g = tile(t);
        const int X0 = g.X0, y0 = g.Y0, ya = g.ya, wa = g.wa, nwd = g.nwd;
        const unsigned long long ma = ~0ull << (g.xa & 63), mb = ~0ull >> (63 - (g.xb & 63));
        unsigned long long m[NS][3];
        int cnt[NS];
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            m[sl][0] = n[sl][0] & ma;
            m[sl][1] = n[sl][1];
            m[sl][2] = n[sl][2];
            if (nwd == 1) m[sl][0] &= mb;
            if (nwd == 2) m[sl][1] &= mb;
            if (nwd == 3) m[sl][2] &= mb;
            cnt[sl] = __popcll(m[sl][0]) + __popcll(m[sl][1]) + __popcll(m[sl][2]);
        }
        // the prefetched words are consumed before new loads are issued
        asm volatile("" ::"v"(cnt[0]), "v"(cnt[1]), "v"(cnt[2]) : "memory");
        const int x = X0 + col;
        float sv[HL];
#pragma unroll
        for (int r = 0; r < HL; ++r) {
            const int y = y0 + rg * HL + r;
            sv[r] = (x < W && y < H) ? S[(size_t)y * W + x] : 0.0f;
        }
        fetch(t + tstep);

        // row-major prefix of the halo row counts
        int excl[NS], total = 0;
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            int tot;
            const int e = wave_excl_small(cnt[sl], tot);
            excl[sl] = total + e;
            total += tot;
        }
        // first row start at or after v (row order: slot-major, then lane)
        auto first_at_least = [&](int v) {
#pragma unroll
            for (int sl = 0; sl < NS; ++sl) {
                const unsigned long long b = __ballot(excl[sl] >= v);
                if (b) return __builtin_amdgcn_readlane(excl[sl], __builtin_ctzll(b));
            }
            return total;
        };

        const int lb = opaque_lane(tbase + ((X0 + col + padx) * stride + (y0 + rg * HL + pady)) * 4);
        vec_t acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = (vec_t)(0.0f);
        const int npass = (total + capp - 1) / capp;
        for (int pass = 0; pass < npass; ++pass) {
            int sp = 0, ep = total;
            if (npass > 1) {
                sp = first_at_least(pass * capp);
                if (pass + 1 < npass) ep = first_at_least((pass + 1) * capp);
            }
#pragma unroll
            for (int sl = 0; sl < NS; ++sl) {
                if (cnt[sl] > 0 && excl[sl] >= sp && excl[sl] < ep) {
                    const int py = ya + 64 * sl + lane;
                    const int c = (py - pady) & (VEC - 1);
                    const int rowterm = c * copy_elems * 4 - (py - c) * 4;
                    int o = excl[sl] - sp;
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        unsigned long long mj = m[sl][j];
                        const int xw = (wa + j) * 64;
                        while (mj) {
                            const int b = __builtin_ctzll(mj);
                            mj &= mj - 1ull;
                            list[o++] = rowterm - (xw + b) * stride * 4;
                        }
                    }
                }
            }
            // the list writes of all lanes complete before the wave reads them
            __builtin_amdgcn_s_waitcnt(0xC07F);
            asm volatile("" ::: "memory");
            const int hi = ep - sp;
            int i = 0;
            const int4 *list4 = reinterpret_cast<const int4 *>(list);
            for (; i + 8 <= hi; i += 8) {
                const int4 ea = list4[i >> 2];
                const int4 eb = list4[(i >> 2) + 1];
                const int a[8] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
                vec_t v[8][NQ];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const lds_vec sp8 = reinterpret_cast<lds_vec>((uint32_t)(lb + a[u]));
#pragma unroll
                    for (int q = 0; q < NQ; ++q) v[u][q] = sp8[q];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q) acc[q] += v[u][q];
                }
            }
            for (; i < hi; ++i) gather_one<NQ>(acc, lb + list[i]);
            // this pass's reads precede the next pass's writes
            asm volatile("" ::: "memory");
        }

        if (x < W) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
#pragma unroll
                for (int j = 0; j < VEC; ++j) {
                    const int y = y0 + rg * HL + q * VEC + j;
                    if (y < H) P[(size_t)y * W + x] = sv[q * VEC + j] + acc[q][j];
                }
            }
        }
    }
}

// Stamp copies for the source-list gather (see ListCfg): copy c holds
// phi(dx, dy) at (dx + padx)*stride + (dy + pady + c); FP64 value rounded once.
// (each copy occupies copy_elems >= ncols*stride floats; the tail is zero)
__global__ void k_phi_copies(float *tab, int vec, int copy_elems, int ncols, int stride, int padx,
                             int pady, int R, double k, double alpha)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= vec * copy_elems) return;
    const int c = i / copy_elems, rem = i - c * copy_elems;
    double v = 0.0;
    if (rem < ncols * stride) {
        const int ci = rem / stride, ri = rem - ci * stride;
        const int dx = ci - padx, dy = ri - c - pady;
        if (abs(dx) <= R && abs(dy) <= R && (dx != 0 || dy != 0))
            v = k * pow(sqrt((double)dx * dx + (double)dy * dy), alpha);
    }
    tab[i] = (float)v;
}

// ---- occupancy ----------------------------------------------------------------------

__global__ void k_occ_init(const int32_t *__restrict__ pos, int N, unsigned long long *occ, int wpr,
                           int W, int32_t *__restrict__ owner, unsigned long long *ctr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = i < N ? pos[i] : -1;
    if (p >= 0) {
        const int y = p / W, x = p - y * W;
        atomicOr(&occ[(size_t)y * wpr + (x >> 6)], 1ull << (x & 63));
        owner[p] = i;
    }
    block_sum_add(p >= 0 ? 1u : 0u, ctr, kLive);
}

// ---- bin + decide + claim (k-2, k-3 registration) --------------------------------------
//
// Binning is a counting sort whose bins are the 64-su row words of the
// occupancy bitmap: each wave takes `chunk` consecutive words, the per-word
// counts are popcounts, a wave prefix sum gives each word's first slot, and
// every lane scatters its word's su indices (ascending x) into a wave-private
// LDS list.  The wave then decides for the listed pedestrians 64 at a time,
// so neighbouring lanes work on neighbouring su.

constexpr int kDecideThreads = 256;

__global__ __launch_bounds__(kDecideThreads) void k_decide_claim(
    int chunk, const unsigned long long *__restrict__ occ, int wpr, int W, int H,
    const int32_t *__restrict__ owner, const float *__restrict__ P, float phi_axial,
    float phi_diag, unsigned long long seed, int32_t *__restrict__ target,
    unsigned long long *__restrict__ key, uint8_t *__restrict__ flags, unsigned long long *claim,
    unsigned long long *ctr)
{
    extern __shared__ int32_t list_raw[];
    const int lane = (int)lane_id();
    const int wv = threadIdx.x >> 6;
    int32_t *list = list_raw + (size_t)wv * chunk * 64;
    const size_t nwords = (size_t)wpr * H;
    const size_t w = ((size_t)blockIdx.x * (kDecideThreads / 64) + wv) * chunk + lane;
    unsigned long long m = 0;
    if (lane < chunk && w < nwords) m = occ[w];
    const int cntl = __popcll(m);
    int total;
    int o = wave_excl_small(cntl, total);
    if (m) {
        const int y = (int)(w / wpr);
        const int xb = (int)(w % wpr) * 64;
        while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1ull;
            list[o++] = y * W + xb + b;
        }
    }
    // the list is private to the wave: its writes complete before it is read
    __builtin_amdgcn_s_waitcnt(0xC07F);
    asm volatile("" ::: "memory");
    const unsigned long long t = ctr[0];
    unsigned int movers = 0, ties = 0;
    for (int base = 0; base < total; base += 64) {
        const int k = base + lane;
        if (k >= total) break;
        const int p = list[k];
        const int i = owner[p];
        const int y = p / W, x = p - y * W;
        float lo = P[p], lo2 = INFINITY;
        int best = 0;
#pragma unroll
        for (int d = 1; d <= 8; ++d) {
            const int nx = x + kDirX[d], ny = y + kDirY[d];
            if (nx >= 0 && ny >= 0 && nx < W && ny < H) {
                const unsigned long long wbits = occ[(size_t)ny * wpr + (nx >> 6)];
                const float pc = P[(size_t)ny * W + nx];
                // P is +inf on obstacle su
                if (!((wbits >> (nx & 63)) & 1ull) && pc < INFINITY) {
                    const float u = pc - ((d & 1) ? phi_axial : phi_diag);
                    if (u < lo) {
                        lo2 = lo;
                        lo = u;
                        best = d;
                    } else if (u < lo2) {
                        lo2 = u;
                    }
                }
            }
        }
        const float scale = fmaxf(fmaxf(fabsf(lo), fabsf(lo2)), 1.0f);
        const bool tied = lo2 < INFINITY && (lo2 - lo) <= 1e-5f * scale;
        int tgt = p;
        bool mover = false;
        if (best != 0) {
            tgt = (y + kDirY[best]) * W + (x + kDirX[best]);
            const uint32_t r = philox_w0((uint32_t)i, (uint32_t)t, (uint32_t)(t >> 32), 0u,
                                         (uint32_t)seed, (uint32_t)(seed >> 32));
            const unsigned long long kk = ((unsigned long long)r << 32) | (uint32_t)i;
            atomicMin(&claim[tgt], kk);
            key[i] = kk;
            mover = true;
        }
        target[i] = tgt;
        flags[i] = (uint8_t)((mover ? kMover : 0u) | (tied ? kTied : 0u));
        movers += mover;
        ties += tied;
    }
    block_sum_add(movers, ctr, kMovers);
    block_sum_add(ties, ctr, kTied);
}

// ---- commit (k-4 moves, exits) -------------------------------------------------------

__global__ __launch_bounds__(256) void k_commit(int N, int W, int32_t *__restrict__ pos,
                                                int32_t *__restrict__ target,
                                                const unsigned long long *__restrict__ key,
                                                uint8_t *__restrict__ flags,
                                                unsigned long long *claim, unsigned long long *occ,
                                                int wpr, int32_t *owner,
                                                const uint8_t *__restrict__ exitm,
                                                unsigned long long *ctr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool was_live = false, won = false, left = false;
    if (i < N) {
        const int p = pos[i];
        if (p < 0) {
            target[i] = -1;
            flags[i] = 0;
        } else {
            was_live = true;
            const uint8_t f = flags[i];
            if (f & kMover) {
                const int tgt = target[i];
                const unsigned long long kk = key[i];
                // the winner is the only registrant that finds its own key; it
                // also resets the word, which losers then read as "not mine"
                if (claim[tgt] == kk) {
                    won = true;
                    claim[tgt] = ~0ull;
                    const int y = p / W, x = p - y * W;
                    atomicAnd(&occ[(size_t)y * wpr + (x >> 6)], ~(1ull << (x & 63)));
                    owner[p] = -1;
                    if (exitm[tgt]) {
                        left = true;
                        pos[i] = -1;
                    } else {
                        const int ty = tgt / W, tx = tgt - ty * W;
                        atomicOr(&occ[(size_t)ty * wpr + (tx >> 6)], 1ull << (tx & 63));
                        owner[tgt] = i;
                        pos[i] = tgt;
                    }
                    flags[i] = f | kWon;
                }
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctr[0], 1ull);
    block_sum_add(was_live ? 1u : 0u, ctr, kPedSteps);
    block_sum_add(won ? 1u : 0u, ctr, kMoved);
    block_sum_add(left ? 1u : 0u, ctr, kEvacuated);
    block_delta_add(left ? -1 : 0, ctr, kLive);
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

inline unsigned int blocks_for(size_t n, unsigned int bs, unsigned int cap = 65535u * 16u)
{
    size_t b = (n + bs - 1) / bs;
    if (b == 0) b = 1;
    return (unsigned int)(b > cap ? cap : b);
}

template <typename T, int TW, int HL, bool ADD_S>
hipError_t sup_launch(const SupCfg &c, const unsigned long long *bits, int wpr, const T *tab,
                      const float *S, T *outT, float *outP, int W, int H, hipStream_t st)
{
    constexpr int TH = (64 / TW) * HL;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int n_tiles = tiles_x * tiles_y;
    const int want = (n_tiles + kSupThreads / 64 - 1) / (kSupThreads / 64);
    const int grid = want < c.grid ? want : c.grid;
    hipLaunchKernelGGL((k_superpose<T, TW, HL, ADD_S>), dim3(grid > 0 ? grid : 1), dim3(kSupThreads),
                       c.lds_bytes, st, bits, wpr, tab, c.ncols * c.stride, c.stride, c.padx,
                       c.pady, c.radius, S, outT, outP, W, H, tiles_x, n_tiles);
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

hipError_t launch_mask_to_bits(const uint8_t *mask, unsigned long long *bits, int W, int H, int wpr,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_mask_to_bits, dim3(blocks_for((size_t)wpr * H, 256, 8192)), dim3(256), 0,
                       st, mask, bits, W, H, wpr);
    return hipGetLastError();
}

hipError_t launch_phi_table_f32(float *tab, const SupCfg &c, double k, double alpha, hipStream_t st)
{
    const int n = c.ncols * c.stride;
    hipLaunchKernelGGL(k_phi_table<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st, tab, c.ncols,
                       c.nrows, c.stride, c.padx, c.pady, c.radius, k, alpha);
    return hipGetLastError();
}

hipError_t launch_phi_table_f64(double *tab, const SupCfg &c, double k, double alpha,
                                hipStream_t st)
{
    const int n = c.ncols * c.stride;
    hipLaunchKernelGGL(k_phi_table<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st, tab,
                       c.ncols, c.nrows, c.stride, c.padx, c.pady, c.radius, k, alpha);
    return hipGetLastError();
}

hipError_t launch_bfs_init(const uint8_t *obst, const uint8_t *exitm, int32_t *D, int32_t *frontier,
                           unsigned int *cnt, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_bfs_init, dim3(blocks_for(n, 256)), dim3(256), 0, st, obst, exitm, D,
                       frontier, cnt, n);
    return hipGetLastError();
}

hipError_t launch_bfs_levels(const uint8_t *obst, int32_t *D, int32_t *fa, int32_t *fb,
                             unsigned int *cnt, int W, int H, int level0, int levels, int grid,
                             hipStream_t st)
{
    for (int L = level0; L < level0 + levels; ++L) {
        const int32_t *fin = (L & 1) ? fb : fa;
        int32_t *fout = (L & 1) ? fa : fb;
        hipLaunchKernelGGL(k_bfs_expand, dim3(grid), dim3(256), 0, st, obst, D, fin, fout, cnt, W,
                           H, L);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_count_unreachable(const uint8_t *obst, const int32_t *D, int n,
                                    unsigned long long *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_unreachable, dim3(blocks_for(n, 256)), dim3(256), 0, st, obst, D, n,
                       out);
    return hipGetLastError();
}

hipError_t set_superpose_lds_limit(size_t f64_bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_superpose<double, 8, 1, false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)f64_bytes);
}

// ---- source-list gather: configuration and launch ------------------------------------

namespace {

// Most lanes of one LDS read of a source's column slice that share a bank:
// lane l (column l % tw, row group l / tw) reads the hl contiguous dwords at
// col*stride + rg*hl.  The LDS serves 256 bytes per clock, so 64 / hl lanes
// form one pass.
int bank_degree(int tw, int hl, int stride)
{
    const int lanes = 64 / hl;
    int worst = 0;
    for (int p = 0; p < 64; p += lanes) {
        int hits[64] = {0};
        for (int l = p; l < p + lanes && l < 64; ++l) {
            const int col = l % tw, rg = l / tw;
            const int a = col * stride + rg * hl;
            for (int j = 0; j < hl; ++j) ++hits[(a + j) % 64];
        }
        for (int b = 0; b < 64; ++b) worst = hits[b] > worst ? hits[b] : worst;
    }
    return worst;
}

}  // namespace

ListCfg make_list_cfg(int radius, int tw, int hl, int vec, int nw, int list_cap, bool wave_lists)
{
    ListCfg c;
    c.wave_lists = wave_lists;
    c.tw = tw;
    c.hl = hl;
    c.vec = vec;
    c.nw = nw;
    c.g = 64 / tw;
    c.th = c.g * hl;
    c.wt = nw * c.th;
    c.radius = radius;
    c.padx = radius + tw;
    c.pady = radius + c.th - 1;
    c.ncols = 2 * c.padx + 1;
    c.nrows = 2 * c.pady + 1;
    const int min_s = c.nrows + vec - 1;
    int best = -1, best_deg = 1 << 30;
    for (int s = min_s; s < min_s + 64; ++s) {
        if (s % vec != 0) continue;  // aligned VEC-wide reads
        const int d = bank_degree(tw, hl, s);
        if (d < best_deg) {
            best_deg = d;
            best = s;
        }
        if (d == 1) break;
    }
    c.stride = best;
    c.copy_elems = (c.ncols * c.stride + 3) & ~3;  // copies start 16-byte aligned
    c.max_row = tw + 2 * radius;
    c.list_cap = list_cap;
    if (wave_lists) {
        // per wave: halo of TH + 2R rows (at most 3 x 64 lanes), list of list_cap
        c.halo_rows = c.th + 2 * radius;
        c.lds_bytes = (size_t)vec * c.copy_elems * 4 + (size_t)nw * list_cap * 4;
    } else {
        c.halo_rows = c.wt + 2 * radius;
        c.lds_bytes = (size_t)vec * c.copy_elems * 4 + (size_t)list_cap * 4 +
                      (size_t)(c.halo_rows + 1) * 4;
    }
    return c;
}

ListCfg pick_list_cfg(int radius, size_t max_lds)
{
    // one list per workgroup strip, 16-column strips, one aligned 8-byte read
    // per source and lane (conflict-free banks); two workgroups per CU are
    // preferred, smaller lists and workgroups if LDS is short
    const int shapes[][4] = {{16, 2, 2, 8}, {16, 2, 2, 4}};
    ListCfg best;
    for (int i = 0; i < 2; ++i) {
        const int *sh = shapes[i];
        for (int cap = 4096; cap >= 512; cap /= 2) {
            ListCfg t = make_list_cfg(radius, sh[0], sh[1], sh[2], sh[3], cap, false);
            if (cap < 2 * t.max_row || t.halo_rows > 64 * sh[3]) break;
            if (t.lds_bytes <= max_lds / 2) return t;
            if (t.lds_bytes <= max_lds && best.lds_bytes == 0) best = t;
        }
    }
    return best;
}

hipError_t launch_phi_copies(float *tab, const ListCfg &c, double k, double alpha, hipStream_t st)
{
    const int n = c.vec * c.copy_elems;
    hipLaunchKernelGGL(k_phi_copies, dim3(blocks_for(n, 256)), dim3(256), 0, st, tab, c.vec,
                       c.copy_elems, c.ncols, c.stride, c.padx, c.pady, c.radius, k, alpha);
    return hipGetLastError();
}

namespace {

template <int TW, int HL, int VEC, int NW>
hipError_t field_wave_launch(const ListCfg &c, const unsigned long long *bits, int wpr,
                             const float *tab, const float *S, float *P, int W, int H,
                             hipStream_t st, const LaunchEvents *ev)
{
    constexpr int TH = (64 / TW) * HL;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int n_tiles = tiles_x * tiles_y;
    const int want = (n_tiles + NW - 1) / NW;
    const int grid = want < c.grid ? want : c.grid;
    return launch(k_field_wave<TW, HL, VEC, NW>, dim3(grid > 0 ? grid : 1), dim3(NW * 64),
                  c.lds_bytes, st, ev, bits, wpr, tab, c.copy_elems, c.stride, c.padx, c.pady,
                  c.radius, c.list_cap, c.max_row, S, P, W, H, tiles_x, n_tiles);
}

template <int TW, int HL, int VEC, int NW>
hipError_t field_list_launch(const ListCfg &c, const unsigned long long *bits, int wpr,
                             const float *tab, const float *S, float *P, int W, int H,
                             hipStream_t st, const LaunchEvents *ev)
{
    if (c.wave_lists)
        return field_wave_launch<TW, HL, VEC, NW>(c, bits, wpr, tab, S, P, W, H, st, ev);
    constexpr int WT = NW * (64 / TW) * HL;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + WT - 1) / WT;
    const int n_tiles = tiles_x * tiles_y;
    const int grid = n_tiles < c.grid ? n_tiles : c.grid;
    return launch(k_field_list<TW, HL, VEC, NW>, dim3(grid > 0 ? grid : 1), dim3(NW * 64),
                  c.lds_bytes, st, ev, bits, wpr, tab, c.copy_elems, c.stride, c.padx, c.pady,
                  c.radius, c.list_cap, c.max_row, S, P, W, H, tiles_x, n_tiles);
}

}  // namespace

#define SF_LIST_SHAPES(X)                                                                     \
    X(16, 2, 2, 4) X(16, 2, 2, 8) X(16, 4, 2, 4) X(16, 4, 2, 8) X(16, 4, 4, 4) X(16, 4, 4, 8)    \
    X(32, 2, 2, 4) X(32, 2, 2, 8) X(32, 4, 2, 4) X(32, 4, 4, 4) X(8, 4, 4, 4) X(8, 2, 2, 4)

bool list_shape_compiled(int tw, int hl, int vec, int nw)
{
#define SF_KNOWN(a, b, v, n) \
    if (tw == a && hl == b && vec == v && nw == n) return true;
    SF_LIST_SHAPES(SF_KNOWN)
#undef SF_KNOWN
    return false;
}

hipError_t set_field_list_lds_limit(size_t bytes)
{
    hipError_t e = hipSuccess;
#define SF_SET(a, b, v, n)                                                                        \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_field_list<a, b, v, n>),         \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);          \
    if (e != hipSuccess) return e;                                                            \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_field_wave<a, b, v, n>),         \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);          \
    if (e != hipSuccess) return e;
    SF_LIST_SHAPES(SF_SET)
#undef SF_SET
    return e;
}

hipError_t launch_field_list(const ListCfg &c, const unsigned long long *bits, int wpr,
                             const float *tab, const float *S, float *P, int W, int H,
                             hipStream_t st, const LaunchEvents *ev)
{
#define SF_DISPATCH(a, b, v, n)                                                                   \
    if (c.tw == a && c.hl == b && c.vec == v && c.nw == n)                                      \
        return field_list_launch<a, b, v, n>(c, bits, wpr, tab, S, P, W, H, st, ev);
    SF_LIST_SHAPES(SF_DISPATCH)
#undef SF_DISPATCH
    return hipErrorInvalidValue;
}

hipError_t launch_superpose_f64(const SupCfg &c, const unsigned long long *bits, int wpr,
                                const double *tab, double *out, int W, int H, hipStream_t st)
{
    if (c.tw == 8 && c.hl == 1)
        return sup_launch<double, 8, 1, false>(c, bits, wpr, tab, nullptr, out, nullptr, W, H, st);
    return hipErrorInvalidValue;
}

hipError_t launch_static_S(const int32_t *D, const double *O, const uint8_t *obst, double w_dest,
                           float *S, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_static_S, dim3(blocks_for(n, 256)), dim3(256), 0, st, D, O, obst, w_dest,
                       S, n);
    return hipGetLastError();
}

hipError_t launch_occ_init(const int32_t *pos, int N, unsigned long long *occ, int wpr, int W,
                           int32_t *owner, unsigned long long *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_occ_init, dim3(blocks_for(N, 256)), dim3(256), 0, st, pos, N, occ, wpr, W,
                       owner, ctr);
    return hipGetLastError();
}

int pick_decide_chunk(int W, int H, int N)
{
    // a wave of `chunk` words holds chunk * 64 * N / (W*H) pedestrians on
    // average: aim at about one per lane
    const double su_per_ped = (double)W * H / (N > 0 ? N : 1);
    int c = 4;
    while (c < 64 && c * 2 <= su_per_ped) c *= 2;
    return c;
}

hipError_t launch_decide_claim(int chunk, const unsigned long long *occ, int wpr, int W, int H,
                               const int32_t *owner, const float *P, float phi_axial,
                               float phi_diag, unsigned long long seed, int32_t *target,
                               unsigned long long *key, uint8_t *flags, unsigned long long *claim,
                               unsigned long long *ctr, hipStream_t st, const LaunchEvents *ev)
{
    const size_t nwords = (size_t)wpr * H;
    const size_t per_block = (size_t)(kDecideThreads / 64) * chunk;
    const size_t lds = (size_t)(kDecideThreads / 64) * chunk * 64 * sizeof(int32_t);
    return launch(k_decide_claim, dim3(blocks_for(nwords, (unsigned)per_block)),
                  dim3(kDecideThreads), lds, st, ev, chunk, occ, wpr, W, H, owner, P, phi_axial,
                  phi_diag, seed, target, key, flags, claim, ctr);
}

hipError_t launch_commit(int N, int W, int32_t *pos, int32_t *target, const unsigned long long *key,
                         uint8_t *flags, unsigned long long *claim, unsigned long long *occ,
                         int wpr, int32_t *owner, const uint8_t *exitm, unsigned long long *ctr,
                         hipStream_t st, const LaunchEvents *ev)
{
    return launch(k_commit, dim3(blocks_for(N, 256)), dim3(256), 0, st, ev, N, W, pos, target, key,
                  flags, claim, occ, wpr, owner, exitm, ctr);
}

}  // namespace sf
