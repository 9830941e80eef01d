/*
 * FP64 CPU oracle of the discrete social-field pedestrian step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product library never does, and
 * it shares no code, header, table or helper with the HIP path.
 *
 * What it computes (Yu, Zhu, Wu, Zhang, "Improved OpenCL-based Implementation
 * of Social Field Pedestrian Model"):
 *   - the discrete model of section 2: a grid of space units (su), one centre
 *     su per pedestrian, at most one su of movement per tick (v_max = 1), so a
 *     pedestrian's candidates are its own su and its 8 Moore neighbours;
 *   - the fields of section 2: a static attractive field of the openings
 *     (destination field: 8-neighbour unit-cost BFS distance to the exit set),
 *     a static repulsive field of the obstacles, and the recurrent repulsive
 *     field of every pedestrian over its square window, superposed linearly
 *     (the write-back of k-5, section 3.1 and Algorithms 2/3: only the total
 *     of the contributions matters);
 *   - the tick of Algorithm 1: k-2 each pedestrian picks its next su, k-3 an
 *     election among the at most 8 pedestrians registered for an unoccupied
 *     su picks one occupant (s-2), k-4 winners move, losers stay;
 *   - openings remove the pedestrians that enter them (Fig. 6 caption, task 11).
 *
 * Readings taken where the paper is silent (listed in the design notes):
 *   field law      phi(d) = fl32(k * |d|_2^alpha) for 0 < |d|_inf <= R,
 *                  phi(0) = 0 (the paper quotes k = 1, alpha = -0.5 for the
 *                  7x7 recurrent repulsive field of Fig. 1 and states a 1x1
 *                  geometry has no fan-out, i.e. no strength at the field's own
 *                  centre); strengths are FP32 numbers, as in the paper's
 *                  float caches (Algorithms 2 and 3);
 *   sums           every field is summed in FP64; for the laws and radii used
 *                  here each sum of FP32 strengths is exact (their exponents
 *                  span few binades), so the summation order does not matter;
 *   regulation     identity; no local-density term; P = w_D*D + O + Phi;
 *   candidates     own su, plus each Moore neighbour that is inside the grid,
 *                  not an obstacle and unoccupied at the start of the tick;
 *   choice         minimum of u(y) = P(y) - phi(y - x) (own field removed),
 *                  lowest direction index on exact ties; the decision is
 *                  taken on FP32 values fl32(fl32(P) - fl32(phi)), the
 *                  paper's field precision;
 *   near tie       the two smallest FP64 u differ by <= 1e-5*max(|u1|,|u2|,1);
 *   election       minimum key = philox(id, t).x * 2^32 + id, where philox is
 *                  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *                  counter (id, t_lo, t_hi, 0) and key (seed_lo, seed_hi).
 *
 * The experiments of section 5 run on a periodic boundary with pedestrian
 * flows in 1, 2, 4 or 8 directions and no openings; the readings for them:
 *   periodic       both axes wrap (a torus): field windows, candidates and
 *                  positions are taken modulo W and H; no exits, so no
 *                  destination field (D = 0);
 *   heading        pedestrian i may carry a heading h_i (one of the eight
 *                  directions e1..e8, 0 = none): the candidate reached by
 *                  move e_d (d = 1..8) gets -w_h * cos(angle(e_h, e_d)) added
 *                  to its value, staying gets 0.  The direction list turns by
 *                  45 degrees per index, so the angle is 45 * min(|h - d|,
 *                  8 - |h - d|) degrees and the cosine is one of 1, 1/sqrt2, 0,
 *                  -1/sqrt2, -1; the FP32 decision uses fl32(w_h) and
 *                  fl32(w_h / sqrt2) with the cosine's sign.
 *   walk period    pedestrian i may carry a walk period p_i >= 1 (section 5:
 *                  speed 1/p_i su per tick): it acts only on ticks t with
 *                  (t + i) mod p_i = 0; on the others it stays without
 *                  deciding or registering (it still occupies its su and
 *                  spreads its field).
 *
 * Pedestrians larger than one su (section 2: odd width and height, so one su
 * is the centre; the experiments of Table VI):
 *   body           a bw x bh block of su centred on the pedestrian's su
 *                  (bw, bh odd, the same for every pedestrian of a scene);
 *                  bodies lie in the grid (or wrap on a torus), cover no
 *                  obstacle and no exit, and never overlap;
 *   field          the pedestrian's field radiates from its centre su;
 *   candidates     move e is a candidate if the body shifted by e lies in
 *                  the grid, covers no obstacle and no su of another body at
 *                  the start of the tick; the value is taken at the shifted
 *                  centre as for one su;
 *   registration   a mover registers for every su its shifted body covers
 *                  and its current body does not (the su it enters);
 *   election       it wins if its key is the smallest at every su it
 *                  registered for; losers stay;
 *   openings       a winner whose shifted body covers an exit su leaves.
 * With bw = bh = 1 these are exactly the one-su rules above.
 *
 * Direction list: e0 = (0,0) stay, e1 = (1,0), e2 = (1,1), e3 = (0,1),
 * e4 = (-1,1), e5 = (-1,0), e6 = (-1,-1), e7 = (0,-1), e8 = (1,-1); x is the
 * column (east +), y the row (south +); linear index c = y*W + x.
 *
 * Parity pins: see the oracle tests (library routines, closed forms,
 * invariants and hand-worked scenes).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const int DIR_X[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
static const int DIR_Y[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};

/* ---- field law ---------------------------------------------------------- */

/* phi at offset (dx, dy) for a field of half-width R (0 outside the window).
 * The strength is an FP32 number: the law is evaluated in FP64 and rounded
 * once to FP32, the precision of the paper's field caches (the float cache[]
 * of Algorithm 2 and float s[K] of Algorithm 3).  Returned as a double. */
double orc_phi(int dx, int dy, int R, double k, double alpha)
{
    int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
    if (adx > R || ady > R) return 0.0;
    if (dx == 0 && dy == 0) return 0.0;
    double dist = sqrt((double)dx * dx + (double)dy * dy);
    return (double)(float)(k * pow(dist, alpha));
}

/* Full (2R+1)^2 stamp, row-major [dy+R][dx+R]. */
void orc_phi_table(int R, double k, double alpha, double *out)
{
    int n = 2 * R + 1;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx)
            out[(dy + R) * n + (dx + R)] = orc_phi(dx, dy, R, k, alpha);
}

/* ---- destination field: BFS distance to the exits ----------------------- */

/* D[c] = number of 8-neighbour unit steps from c to the nearest exit su over
 * non-obstacle su; -1 on obstacles and on su that cannot reach an exit.
 * Returns the number of non-obstacle su that cannot reach an exit. */
int64_t orc_bfs_distance(int W, int H, const uint8_t *obst, const uint8_t *exitm,
                         int32_t *D)
{
    int64_t n = (int64_t)W * H;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t head = 0, tail = 0;
    for (int64_t c = 0; c < n; ++c) {
        D[c] = -1;
        if (exitm[c] && !obst[c]) {
            D[c] = 0;
            queue[tail++] = (int32_t)c;
        }
    }
    while (head < tail) {
        int32_t c = queue[head++];
        int x = c % W, y = c / W;
        for (int d = 1; d <= 8; ++d) {
            int nx = x + DIR_X[d], ny = y + DIR_Y[d];
            if (nx < 0 || ny < 0 || nx >= W || ny >= H) continue;
            int64_t nc = (int64_t)ny * W + nx;
            if (obst[nc] || D[nc] >= 0) continue;
            D[nc] = D[c] + 1;
            queue[tail++] = (int32_t)nc;
        }
    }
    free(queue);
    int64_t unreachable = 0;
    for (int64_t c = 0; c < n; ++c)
        if (!obst[c] && D[c] < 0) ++unreachable;
    return unreachable;
}

/* ---- superposed source field -------------------------------------------- */

/* out[c] = sum over source su s (src[s] != 0) of phi(c - s), for every su c of
 * the grid.  Each source spreads its window; contributions outside the grid
 * are dropped, or wrap around when `periodic`.  Plain scatter in source raster
 * order, FP64. */
void orc_source_field(int W, int H, const uint8_t *src, int R, double k, double alpha,
                      int periodic, double *out)
{
    int64_t n = (int64_t)W * H;
    int m = 2 * R + 1;
    double *tab = (double *)malloc(sizeof(double) * (size_t)m * m);
    orc_phi_table(R, k, alpha, tab);
    for (int64_t c = 0; c < n; ++c) out[c] = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        if (!src[s]) continue;
        int sx = (int)(s % W), sy = (int)(s / W);
        for (int dy = -R; dy <= R; ++dy) {
            int y = sy + dy;
            if (periodic)
                y = ((y % H) + H) % H;
            else if (y < 0 || y >= H)
                continue;
            for (int dx = -R; dx <= R; ++dx) {
                int x = sx + dx;
                if (periodic)
                    x = ((x % W) + W) % W;
                else if (x < 0 || x >= W)
                    continue;
                out[(int64_t)y * W + x] += tab[(dy + R) * m + (dx + R)];
            }
        }
    }
    free(tab);
}

/* The same field computed by `nthreads` POSIX threads, thread j owning a band
 * of output rows: it scatters every source within R rows of its band, but
 * writes only the su of its band.  Each su receives the same terms as in the
 * serial scatter; every sum of FP32 strengths is exact in FP64, so the result
 * is the serial one bit for bit. */
typedef struct {
    int W, H, R, periodic, m, y0, y1;
    const uint8_t *src;
    const double *tab;
    double *out;
} band_job;

static void *band_scatter(void *arg)
{
    const band_job *j = (const band_job *)arg;
    const int W = j->W, H = j->H, R = j->R, m = j->m;
    for (int64_t c = (int64_t)j->y0 * W; c < (int64_t)j->y1 * W; ++c) j->out[c] = 0.0;
    /* source rows whose windows reach the band (each row once, also when the
     * window wraps around a small torus) */
    int lo = j->y0 - R, hi = j->y1 - 1 + R;
    if (!j->periodic) {
        if (lo < 0) lo = 0;
        if (hi > H - 1) hi = H - 1;
    } else if (hi - lo + 1 > H) {
        lo = 0;
        hi = H - 1;
    }
    for (int ry = lo; ry <= hi; ++ry) {
        const int sy = j->periodic ? ((ry % H) + H) % H : ry;
        for (int sx = 0; sx < W; ++sx) {
            if (!j->src[(int64_t)sy * W + sx]) continue;
            for (int dy = -R; dy <= R; ++dy) {
                int y = sy + dy;
                if (j->periodic)
                    y = ((y % H) + H) % H;
                else if (y < 0 || y >= H)
                    continue;
                if (y < j->y0 || y >= j->y1) continue;
                for (int dx = -R; dx <= R; ++dx) {
                    int x = sx + dx;
                    if (j->periodic)
                        x = ((x % W) + W) % W;
                    else if (x < 0 || x >= W)
                        continue;
                    j->out[(int64_t)y * W + x] += j->tab[(dy + R) * m + (dx + R)];
                }
            }
        }
    }
    return NULL;
}

void orc_source_field_mt(int W, int H, const uint8_t *src, int R, double k, double alpha,
                         int periodic, int nthreads, double *out)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > H) nthreads = H;
    int m = 2 * R + 1;
    double *tab = (double *)malloc(sizeof(double) * (size_t)m * m);
    orc_phi_table(R, k, alpha, tab);
    band_job *jobs = (band_job *)malloc(sizeof(band_job) * (size_t)nthreads);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; ++t) {
        band_job j = {W, H, R, periodic, m, (int)((int64_t)H * t / nthreads),
                      (int)((int64_t)H * (t + 1) / nthreads), src, tab, out};
        jobs[t] = j;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, band_scatter, &jobs[t]);
    band_scatter(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
    free(tab);
}

/* Occupancy mask from positions (pos < 0: evacuated). */
void orc_occupancy(int W, int H, int32_t n_peds, const int32_t *pos, uint8_t *occ)
{
    memset(occ, 0, (size_t)W * H);
    for (int32_t i = 0; i < n_peds; ++i)
        if (pos[i] >= 0) occ[pos[i]] = 1;
}

/* P[c] = w_D*D[c] + O[c] + Phi[c] on non-obstacle su, +inf on obstacles.
 * Phi is the superposed pedestrian field of the live pedestrians, computed
 * by one thread or, with nthreads > 1, by the row-band threads above (the
 * same bits). */
void orc_total_field(int W, int H, const uint8_t *obst, const int32_t *D, const double *O,
                     double w_dest, int32_t n_peds, const int32_t *pos, int R, double k,
                     double alpha, int periodic, int nthreads, double *P)
{
    int64_t n = (int64_t)W * H;
    uint8_t *occ = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    orc_occupancy(W, H, n_peds, pos, occ);
    if (nthreads > 1)
        orc_source_field_mt(W, H, occ, R, k, alpha, periodic, nthreads, P);
    else
        orc_source_field(W, H, occ, R, k, alpha, periodic, P);
    for (int64_t c = 0; c < n; ++c)
        P[c] = obst[c] ? INFINITY : w_dest * (double)D[c] + O[c] + P[c];
    free(occ);
}

/* ---- counter-based generator --------------------------------------------- */

/* Philox4x32-10 of Salmon, Moraes, Dror and Shaw ("Parallel Random Numbers: As
 * Easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications
 * (multipliers 0xD2511F53 and 0xCD9E8D57) mixed with the key, the key being
 * advanced by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Election key of pedestrian `id` at step t. */
uint64_t orc_claim_key(int32_t id, int64_t t, uint64_t seed)
{
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)((uint64_t)t & 0xffffffffu),
                       (uint32_t)((uint64_t)t >> 32), 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    return ((uint64_t)r[0] << 32) | (uint32_t)id;
}

/* ---- one tick ------------------------------------------------------------ */

/* Multiples of 45 degrees between directions h and d (both 1..8). */
static int turn_steps(int h, int d)
{
    int s = h > d ? h - d : d - h;
    return s > 4 ? 8 - s : s;
}

/* Heading term of the move e_d (d = 0: staying) for heading h (0: none), in
 * FP64 and as the FP32 decision sees it. */
static double heading_term64(int h, int d, double w_h)
{
    if (h == 0 || d == 0) return 0.0;
    static const double cosv[5] = {1.0, 0.70710678118654752440, 0.0,
                                   -0.70710678118654752440, -1.0};
    return -w_h * cosv[turn_steps(h, d)];
}

static float heading_term32(int h, int d, double w_h)
{
    if (h == 0 || d == 0) return 0.0f;
    float ca = (float)w_h, cd = (float)(w_h / sqrt(2.0));
    switch (turn_steps(h, d)) {
    case 0: return -ca;
    case 1: return -cd;
    case 2: return 0.0f;
    case 3: return cd;
    default: return ca;
    }
}

/* Whether the body of pedestrian `id` (half-widths a, b) shifted to centre
 * (cx, cy) lies in the grid (bounded) or wraps (periodic), covers no obstacle
 * and no su of another body: owner[c] is the pedestrian whose body covers c,
 * or -1. */
static int body_fits(int W, int H, const uint8_t *obst, const int32_t *owner, int32_t id,
                     int a, int b, int periodic, int cx, int cy)
{
    for (int j = -b; j <= b; ++j)
        for (int i = -a; i <= a; ++i) {
            int x = cx + i, y = cy + j;
            if (periodic) {
                x = ((x % W) + W) % W;
                y = ((y % H) + H) % H;
            } else if (x < 0 || y < 0 || x >= W || y >= H) {
                return 0;
            }
            int64_t c = (int64_t)y * W + x;
            if (obst[c] || (owner[c] >= 0 && owner[c] != id)) return 0;
        }
    return 1;
}

/* Decision of one live pedestrian `id` at su p, given the step-start field P
 * and body map.  Writes the chosen su and whether the two best candidates are
 * a near tie.  phi1 / phi2: the pedestrian's own field at an axial / diagonal
 * neighbour; h, w_h: its heading and the heading weight. */
static void decide_one(int W, int H, const uint8_t *obst, const int32_t *owner, int32_t id,
                       int a, int b, const double *P, double phi_axial, double phi_diag,
                       int periodic, int h, double w_h, int32_t p, int32_t *target, uint8_t *tied)
{
    int x = p % W, y = p / W;
    float best32 = 0.0f;
    int best_dir = -1;
    int64_t best_c = p;
    double u_lo = INFINITY, u_lo2 = INFINITY; /* two smallest FP64 values */
    for (int d = 0; d <= 8; ++d) {
        int nx = x + DIR_X[d], ny = y + DIR_Y[d];
        if (periodic) {
            nx = (nx + W) % W;
            ny = (ny + H) % H;
        }
        if (d > 0) {
            if (nx < 0 || ny < 0 || nx >= W || ny >= H) continue;
            if (!body_fits(W, H, obst, owner, id, a, b, periodic, x + DIR_X[d], y + DIR_Y[d]))
                continue;
        }
        int64_t c = (int64_t)ny * W + nx;
        double own = d == 0 ? 0.0 : ((d & 1) ? phi_axial : phi_diag);
        double u64 = P[c] - own + heading_term64(h, d, w_h);
        float u32 = ((float)P[c] - (float)own) + heading_term32(h, d, w_h);
        if (best_dir < 0 || u32 < best32) {
            best32 = u32;
            best_dir = d;
            best_c = c;
        }
        if (u64 < u_lo) {
            u_lo2 = u_lo;
            u_lo = u64;
        } else if (u64 < u_lo2) {
            u_lo2 = u64;
        }
    }
    *target = (int32_t)best_c;
    double scale = fabs(u_lo);
    if (fabs(u_lo2) > scale) scale = fabs(u_lo2);
    if (scale < 1.0) scale = 1.0;
    *tied = (isfinite(u_lo2) && (u_lo2 - u_lo) <= 1e-5 * scale) ? 1 : 0;
}

/* Body map: owner[c] = the live pedestrian whose body covers c, else -1.
 * Returns 0, or 1 + the first pedestrian whose body leaves a bounded grid or
 * overlaps another body (the map then holds the bodies before it). */
int64_t orc_body_map(int W, int H, int32_t n_peds, const int32_t *pos, int bw, int bh,
                     int periodic, int32_t *owner)
{
    int a = (bw - 1) / 2, b = (bh - 1) / 2;
    for (int64_t c = 0; c < (int64_t)W * H; ++c) owner[c] = -1;
    for (int32_t i = 0; i < n_peds; ++i) {
        if (pos[i] < 0) continue;
        int x = pos[i] % W, y = pos[i] / W;
        for (int j = -b; j <= b; ++j)
            for (int q = -a; q <= a; ++q) {
                int sx = x + q, sy = y + j;
                if (periodic) {
                    sx = ((sx % W) + W) % W;
                    sy = ((sy % H) + H) % H;
                } else if (sx < 0 || sy < 0 || sx >= W || sy >= H) {
                    return 1 + (int64_t)i;
                }
                int64_t c = (int64_t)sy * W + sx;
                if (owner[c] >= 0) return 1 + (int64_t)i;
                owner[c] = i;
            }
    }
    return 0;
}

/* Column and row step (-1, 0 or 1) from su p to its neighbour q, across
 * the seam of a torus. */
static int step_dx(int W, int periodic, int32_t p, int32_t q)
{
    int d = q % W - p % W;
    if (periodic && d > 1) d -= W;
    if (periodic && d < -1) d += W;
    return d;
}

static int step_dy(int W, int H, int periodic, int32_t p, int32_t q)
{
    int d = q / W - p / W;
    if (periodic && d > 1) d -= H;
    if (periodic && d < -1) d += H;
    return d;
}

/* Whether pedestrian i acts on tick t (walk period p, NULL or 1: every tick). */
static int acts(const uint8_t *period, int32_t i, int64_t t)
{
    if (!period || period[i] <= 1) return 1;
    return ((uint64_t)t + (uint64_t)i) % period[i] == 0;
}

/* Su of the body of half-widths (a, b) centred at (cx, cy) that the body
 * centred at (ox, oy) does not cover (the centres are at most one su apart,
 * unwrapped); wrapped on a torus.  Writes up to (2a+1)(2b+1) linear indices
 * to out and returns their number. */
static int entered_su(int W, int H, int a, int b, int periodic, int ox, int oy, int cx, int cy,
                      int64_t *out)
{
    int n = 0;
    for (int j = -b; j <= b; ++j)
        for (int i = -a; i <= a; ++i) {
            int x = cx + i, y = cy + j;
            if (x >= ox - a && x <= ox + a && y >= oy - b && y <= oy + b) continue;
            if (periodic) {
                x = ((x % W) + W) % W;
                y = ((y % H) + H) % H;
            }
            out[n++] = (int64_t)y * W + x;
        }
    return n;
}

/* One tick from state (pos, t).
 *   P       [W*H]  the step-start total field (orc_total_field of pos)
 *   heading [N]    headings (NULL: none)
 *   period  [N]    walk periods (NULL: every pedestrian acts every tick)
 *   bw, bh         body width and height (odd; 1, 1: one su per pedestrian)
 *   pos     [N]    in: step-start positions (-1 = evacuated); out: new ones
 *   target  [N]    out: chosen su (own su when staying; -1 when evacuated)
 *   moved   [N]    out: 1 if the pedestrian won its election and moved
 *   tied    [N]    out: 1 if its two best candidates are a near tie
 * Returns the number of pedestrians that left through an exit this tick. */
int64_t orc_step(int W, int H, const uint8_t *obst, const uint8_t *exitm, const double *P,
                 int R, double k, double alpha, int periodic, const uint8_t *heading,
                 double w_h, const uint8_t *period, int bw, int bh, uint64_t seed, int64_t t,
                 int32_t n_peds, int32_t *pos, int32_t *target, uint8_t *moved, uint8_t *tied)
{
    int64_t n = (int64_t)W * H;
    int a = (bw - 1) / 2, b = (bh - 1) / 2;
    int32_t *owner = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orc_body_map(W, H, n_peds, pos, bw, bh, periodic, owner);
    double phi_axial = orc_phi(1, 0, R, k, alpha);
    double phi_diag = orc_phi(1, 1, R, k, alpha);

    /* k-2: every live pedestrian decides on the same step-start state. */
    for (int32_t i = 0; i < n_peds; ++i) {
        moved[i] = 0;
        tied[i] = 0;
        target[i] = -1;
        if (pos[i] < 0) continue;
        if (!acts(period, i, t)) {
            target[i] = pos[i]; /* resting this tick */
            continue;
        }
        decide_one(W, H, obst, owner, i, a, b, P, phi_axial, phi_diag, periodic,
                   heading ? heading[i] : 0, w_h, pos[i], &target[i], &tied[i]);
    }

    /* k-3: per su a mover enters, the registered pedestrian with the smallest
     * key; a mover wins if it holds that key at every su it enters (for one
     * su, its target). */
    int64_t *su = (int64_t *)malloc(sizeof(int64_t) * (size_t)(bw * bh));
    uint64_t *best = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t c = 0; c < n; ++c) best[c] = UINT64_MAX;
    for (int32_t i = 0; i < n_peds; ++i) {
        if (pos[i] < 0 || target[i] == pos[i]) continue;
        uint64_t key = orc_claim_key(i, t, seed);
        int ox = pos[i] % W, oy = pos[i] / W;
        int m = entered_su(W, H, a, b, periodic, ox, oy,
                           ox + step_dx(W, periodic, pos[i], target[i]),
                           oy + step_dy(W, H, periodic, pos[i], target[i]), su);
        for (int q = 0; q < m; ++q)
            if (key < best[su[q]]) best[su[q]] = key;
    }

    /* k-4: winners move (or leave when the body reaches an exit); losers
     * stay.  New positions are written after every winner is known. */
    int64_t left = 0;
    int32_t *newpos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_peds > 0 ? n_peds : 1));
    for (int32_t i = 0; i < n_peds; ++i) {
        newpos[i] = pos[i];
        if (pos[i] < 0 || target[i] == pos[i]) continue;
        uint64_t key = orc_claim_key(i, t, seed);
        int ox = pos[i] % W, oy = pos[i] / W;
        int m = entered_su(W, H, a, b, periodic, ox, oy,
                           ox + step_dx(W, periodic, pos[i], target[i]),
                           oy + step_dy(W, H, periodic, pos[i], target[i]), su);
        int won = 1, at_exit = 0;
        for (int q = 0; q < m; ++q) {
            if (best[su[q]] != key) won = 0;
            if (exitm[su[q]]) at_exit = 1;
        }
        if (!won) continue;
        moved[i] = 1;
        if (at_exit) {
            newpos[i] = -1;
            ++left;
        } else {
            newpos[i] = target[i];
        }
    }
    memcpy(pos, newpos, sizeof(int32_t) * (size_t)(n_peds > 0 ? n_peds : 0));
    free(newpos);
    free(best);
    free(su);
    free(owner);
    return left;
}

/* ---- point evaluation for large grids ------------------------------------ */

/* P at one su from masks (no full-grid pass): w_D*D + sum over obstacle su in
 * the obstacle window + sum over occupied su in the pedestrian window. */
/* Source su row / column of an offset from c: -1 if it falls off a bounded
 * grid, wrapped on a periodic one. */
static int wrap_or_drop(int v, int n, int periodic)
{
    if (periodic) return ((v % n) + n) % n;
    return (v < 0 || v >= n) ? -1 : v;
}

double orc_field_at(int W, int H, const uint8_t *obst, const uint8_t *occ, const int32_t *D,
                    double w_dest, int R, double k, double alpha, int R_obs, double k_obs,
                    double alpha_obs, int periodic, int64_t c)
{
    if (obst[c]) return INFINITY;
    int x = (int)(c % W), y = (int)(c / W);
    double o = 0.0, f = 0.0;
    for (int dy = -R_obs; dy <= R_obs; ++dy) {
        int sy = wrap_or_drop(y - dy, H, periodic);
        if (sy < 0) continue;
        for (int dx = -R_obs; dx <= R_obs; ++dx) {
            int sx = wrap_or_drop(x - dx, W, periodic);
            if (sx < 0) continue;
            if (obst[(int64_t)sy * W + sx]) o += orc_phi(dx, dy, R_obs, k_obs, alpha_obs);
        }
    }
    for (int dy = -R; dy <= R; ++dy) {
        int sy = wrap_or_drop(y - dy, H, periodic);
        if (sy < 0) continue;
        for (int dx = -R; dx <= R; ++dx) {
            int sx = wrap_or_drop(x - dx, W, periodic);
            if (sx < 0) continue;
            if (occ[(int64_t)sy * W + sx]) f += orc_phi(dx, dy, R, k, alpha);
        }
    }
    return w_dest * (double)D[c] + o + f;
}

/* Decision of the pedestrian standing at su p, from point evaluations of the
 * field on its 3x3 neighbourhood.  Same rule as the full-grid tick. */
void orc_decide_at(int W, int H, const uint8_t *obst, const uint8_t *occ, const int32_t *D,
                   double w_dest, int R, double k, double alpha, int R_obs, double k_obs,
                   double alpha_obs, int periodic, int h, double w_h, int32_t p,
                   int32_t *target, uint8_t *tied, double *P9)
{
    double Ploc[9];
    int x = p % W, y = p / W;
    /* field on the 3x3 block around p, stored by direction */
    for (int d = 0; d <= 8; ++d) {
        int nx = wrap_or_drop(x + DIR_X[d], W, periodic);
        int ny = wrap_or_drop(y + DIR_Y[d], H, periodic);
        Ploc[d] = INFINITY;
        if (nx < 0 || ny < 0) continue;
        Ploc[d] = orc_field_at(W, H, obst, occ, D, w_dest, R, k, alpha, R_obs, k_obs,
                               alpha_obs, periodic, (int64_t)ny * W + nx);
    }
    if (P9)
        for (int d = 0; d <= 8; ++d) P9[d] = Ploc[d];
    /* reuse the full-grid rule on a 3x3 window around p */
    uint8_t o3[9];
    int32_t c3[9];
    double P3[9];
    for (int j = 0; j < 9; ++j) {
        o3[j] = 1;
        c3[j] = -1;
        P3[j] = INFINITY;
    }
    for (int d = 0; d <= 8; ++d) {
        int nx = wrap_or_drop(x + DIR_X[d], W, periodic);
        int ny = wrap_or_drop(y + DIR_Y[d], H, periodic);
        if (nx < 0 || ny < 0) continue;
        int64_t nc = (int64_t)ny * W + nx;
        int j = (DIR_Y[d] + 1) * 3 + (DIR_X[d] + 1);
        o3[j] = obst[nc];
        c3[j] = d == 0 ? 0 : (occ[nc] ? 1 : -1);
        P3[j] = Ploc[d];
    }
    int32_t t3;
    decide_one(3, 3, o3, c3, 0, 0, 0, P3, orc_phi(1, 0, R, k, alpha), orc_phi(1, 1, R, k, alpha),
               0, h,
               w_h, 4, &t3, tied);
    int tx = wrap_or_drop(x + t3 % 3 - 1, W, periodic);
    int ty = wrap_or_drop(y + t3 / 3 - 1, H, periodic);
    *target = (int32_t)((int64_t)ty * W + tx);
}

/* ---- the paper's own field path: 8 sects, strength fan-out, K slots -------- */
/*
 * Section 3.1, s-1: each su keeps its field strengths in 8 sects (the shared
 * "3-D image"), and the strength a source puts at su c goes to the sect of
 * the offset d = c - o from the source's su o to c.  For one sect of one su,
 * the set of offsets of the window that land there has the same size wherever
 * the source is: the strength fan-out SF.  Algorithm 2 caches the 8*SF
 * possible strengths of an su and sums them in one pass; Algorithm 3 (with
 * Eq. 1) bounds the cache to K slots: the 8*SF terms, padded with zero
 * strengths to a multiple of K, are split into K blocks of m = 8*SF/K
 * consecutive terms, each block summed into its slot, then the K slots are
 * summed.  The caches are floats, so every sum here is an FP32 sum taken in
 * the stated order.
 *
 * Readings (the sect rule is in figures that are not available):
 *   sect rule      sect(d) = floor(theta / 45 degrees), theta in [0, 360) the
 *                  angle of d from +x (east) toward +y (south); each sect is
 *                  half-open on its far edge.  For a (2R+1)^2 window every
 *                  sect holds R(R+1)/2 offsets, so SF = R(R+1)/2 (the 7x7 field
 *                  of the paper's example has SF = 6).
 *   term order     sect by sect (0..7); within a sect, offsets in row-major
 *                  order (dy ascending, then dx ascending); zero strengths are
 *                  appended at the end to reach a multiple of K.
 *   blocks         block j holds terms j*m .. j*m + m - 1 (Eq. 1 read with the
 *                  block index j*m + i); s[j] is their sequential FP32 sum from
 *                  +0, and the field is ((s[0] + s[1]) + s[2]) + ... in FP32.
 *   image          sect s of su c holds the sequential FP32 sum of that sect's
 *                  terms (for K = 8 the blocks are the sects).
 *   write-back     P = fl32(S + Phi) with Phi the FP32 field, S in FP64.
 *   update         the incremental form of k-4/k-5: the terms are the
 *                  strengths of the su entered (+) and left (-) this tick, and
 *                  the field and image add their block sums: Phi += sum,
 *                  sect += sect sum (FP32).
 */

/* Sect of a nonzero offset: rotate by -90 degrees, (dx, dy) -> (dy, -dx),
 * until it lies in [0, 90) (dx > 0, dy >= 0); two sects per quarter turn. */
int orc_sect(int dx, int dy)
{
    int q = 0;
    while (!(dx > 0 && dy >= 0)) {
        int t = dx;
        dx = dy;
        dy = -t;
        ++q;
    }
    return 2 * q + (dy < dx ? 0 : 1);
}

/* Strength fan-out of a wd x ht field geometry (wd, ht odd): the largest
 * number of window offsets that share one sect (Tables I and II). */
int orc_fan_out(int wd, int ht)
{
    int a = (wd - 1) / 2, b = (ht - 1) / 2, cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0}, best = 0;
    for (int dy = -b; dy <= b; ++dy)
        for (int dx = -a; dx <= a; ++dx)
            if (dx != 0 || dy != 0) ++cnt[orc_sect(dx, dy)];
    for (int s = 0; s < 8; ++s) best = cnt[s] > best ? cnt[s] : best;
    return best;
}

/* The term list of an (2R+1)^2 window in the order above, padded with zero
 * terms to a multiple of K: offsets, strengths, sects (-1 for padding).
 * Returns the padded length n; the arrays hold (2R+1)^2 - 1 + K entries. */
static int sect_terms(int R, double k, double alpha, int K, int *tdx, int *tdy, float *tphi,
                      int *tsect)
{
    int n = 0;
    for (int s = 0; s < 8; ++s)
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx) {
                if ((dx == 0 && dy == 0) || orc_sect(dx, dy) != s) continue;
                tdx[n] = dx;
                tdy[n] = dy;
                tphi[n] = (float)orc_phi(dx, dy, R, k, alpha);
                tsect[n] = s;
                ++n;
            }
    while (n % K != 0) {
        tdx[n] = tdy[n] = 0;
        tphi[n] = 0.0f;
        tsect[n] = -1;
        ++n;
    }
    return n;
}

/* Source bit of su (x, y) - d: 1 if that su is a source (bounded grids have
 * no sources beyond the edge; a torus wraps). */
static int source_at(int W, int H, const uint8_t *src, int periodic, int x, int y)
{
    if (periodic) {
        x = ((x % W) + W) % W;
        y = ((y % H) + H) % H;
    } else if (x < 0 || y < 0 || x >= W || y >= H) {
        return 0;
    }
    return src[(size_t)y * W + x] != 0;
}

/* Algorithm 3 with K slots over every su.  With `minus` == NULL the terms are
 * the strengths of the sources in `plus` (a full field: phi and image are
 * written); otherwise the terms are +strength for `plus` and -strength for
 * `minus` and the block and sect sums are added to phi and image (the
 * update).  image (8 planes of W*H floats) may be NULL.  Returns the padded
 * number of terms, or -1 if K is not one of 2, 4, 8, 16. */
int orc_sect_field(int W, int H, const uint8_t *plus, const uint8_t *minus, int R, double k,
                   double alpha, int periodic, int K, float *phi, float *image)
{
    if (K != 2 && K != 4 && K != 8 && K != 16) return -1;
    const int cap = (2 * R + 1) * (2 * R + 1) - 1 + K;
    int *tdx = malloc(sizeof(int) * cap), *tdy = malloc(sizeof(int) * cap);
    int *tsect = malloc(sizeof(int) * cap);
    float *tphi = malloc(sizeof(float) * cap);
    const int n = sect_terms(R, k, alpha, K, tdx, tdy, tphi, tsect);
    const int m = n / K;
    const size_t plane = (size_t)W * H;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            float slot[16], sect[8];
            for (int j = 0; j < K; ++j) slot[j] = 0.0f;
            for (int s = 0; s < 8; ++s) sect[s] = 0.0f;
            for (int i = 0; i < n; ++i) {
                if (tsect[i] < 0) continue; /* appended zero strength: adds +0 */
                const int sx = x - tdx[i], sy = y - tdy[i];
                float a = 0.0f;
                if (source_at(W, H, plus, periodic, sx, sy)) a = tphi[i];
                if (minus && source_at(W, H, minus, periodic, sx, sy)) a = -tphi[i];
                slot[i / m] = slot[i / m] + a;
                sect[tsect[i]] = sect[tsect[i]] + a;
            }
            float sum = 0.0f;
            for (int j = 0; j < K; ++j) sum = sum + slot[j];
            const size_t c = (size_t)y * W + x;
            if (minus) {
                phi[c] = phi[c] + sum;
                if (image)
                    for (int s = 0; s < 8; ++s) image[s * plane + c] = image[s * plane + c] + sect[s];
            } else {
                phi[c] = sum;
                if (image)
                    for (int s = 0; s < 8; ++s) image[s * plane + c] = sect[s];
            }
        }
    free(tdx);
    free(tdy);
    free(tsect);
    free(tphi);
    return n;
}
