/*
 * libsf -- per-tick update of the discrete social-field pedestrian model on
 * AMD MI355X (gfx950).
 *
 * Model: Yu, Zhu, Wu, Zhang, "Improved OpenCL-based Implementation of Social
 * Field Pedestrian Model".  Section 2 defines the discrete model (a grid of
 * space units, "su"; one centre su per pedestrian; v_max = 1 su per tick),
 * section 3.1 and Algorithm 1 the tick (k-1 .. k-5: decide, register and
 * elect, move, write the field back), Algorithms 2/3 with Eq. 1 the field
 * write-back as a sum of per-source contributions.
 *
 * Readings taken where the paper is silent:
 *   - field law phi(d) = fl32(k*|d|_2^alpha) on the square window
 *     |d|_inf <= R and phi(0) = 0 (Fig. 1 caption: k = 1, alpha = -0.5;
 *     Table I: a 1x1 field has no fan-out); strengths are FP32 numbers, the
 *     precision of the float caches of Algorithms 2 and 3;
 *   - static destination field D = 8-neighbour unit-cost BFS distance to the
 *     exits; static obstacle field O = the same law summed over obstacle su;
 *   - total field P = fl32(S + Phi) with S = w_dest*D + O in FP64 and Phi the
 *     sum of the pedestrians' strengths formed in FP64, +inf on obstacle su.
 *     Every term of a window is a multiple of q = 2^(e - 23), e the exponent
 *     of its smallest nonzero |strength|; sf_create_scene accepts a law (of
 *     the pedestrians, and of the obstacles) only if 4 * sum|strength| over
 *     its window is below 2^53 * q (strengths spread over up to about 2^15),
 *     so that every such sum is an FP64 number and P is the FP64 field
 *     rounded once to FP32 whatever the order of the terms;
 *   - a pedestrian at x chooses, among x and its free in-grid non-obstacle
 *     Moore neighbours y, the minimum of u(y) = P(y) - phi(y - x), lowest
 *     direction index on exact ties; direction order stay, (1,0), (1,1),
 *     (0,1), (-1,1), (-1,0), (-1,-1), (0,-1), (1,-1) (x east, y south);
 *   - the election of k-3 among the <= 8 registrants of an su keeps the
 *     smallest key (Philox4x32-10(counter = (id, t_lo, t_hi, 0),
 *     key = (seed_lo, seed_hi)).word0 << 32) | id; losers stay;
 *   - entering an exit su removes the pedestrian in the same tick;
 *   - section 5's experiments: a periodic boundary (a torus, no exits),
 *     headed flows (a heading adds -w_heading*cos(angle(heading, move)) to a
 *     candidate's value) and walk periods (pedestrian i with period p acts
 *     on ticks t with (t + i) mod p = 0 only).
 *
 * Conventions.
 *   - Grids are row-major, x fastest; linear su index c = y*width + x.
 *   - Every call returns SF_OK (0) or a negative SF_E* code; the message of
 *     the last failure on the calling thread is in sf_last_error().  No C++
 *     exception crosses this boundary.
 *   - Host input arrays are owned by the caller and copied during the call.
 *     Output buffers are owned by the caller.  All device state is owned by
 *     the scene and released by sf_destroy_scene.
 *   - Work of a scene is enqueued on the HIP stream given at creation (NULL =
 *     the null stream) on the device that was current at creation.
 *   - Calls on different scenes may run on different threads; calls on one
 *     scene must not overlap.
 *   - Environment overrides read by sf_create_scene, for tuning only (results
 *     do not depend on them bit for bit): SF_TILE="TWxHLx2xNW[xCAP]" (field
 *     tile shape and source-list capacity), SF_FIELD_BLOCKS_PER_CU (field
 *     workgroups per compute unit) and SF_FIELD_DENSE=0/1 (the dense
 *     small-radius field stencil off / on where the radius allows it).
 */
#ifndef SF_H
#define SF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SF_OK 0
#define SF_EINVAL (-1)       /* bad descriptor or argument                    */
#define SF_ENOMEM (-2)       /* device or host allocation failed              */
#define SF_EDEVICE (-3)      /* a HIP call failed                             */
#define SF_EUNREACHABLE (-4) /* a non-obstacle su has no path to any exit     */

/* Largest field half-width R (pedestrian and obstacle fields) accepted. */
#define SF_MAX_RADIUS 48

/* Largest pedestrian body side in su (odd). */
#define SF_MAX_BODY 15

/* Largest number of pedestrians of one scene (per-pedestrian launches index
 * whole workgroups of 256 with 32-bit ids). */
#define SF_MAX_PEDS (2147483647 - 1023)

typedef struct sf_scene sf_scene; /* opaque, library-owned */

/* Scene description (section 2 grid, pedestrians, field geometry; Algorithm 1
 * tick counter).  All pointers are host pointers, read during
 * sf_create_scene only. */
typedef struct {
    int32_t width, height;    /* grid size in su; width*height < 2^31            */
    const uint8_t *obstacle;  /* [height*width] 1 = obstacle (walls included)    */
    const uint8_t *exit;      /* [height*width] 1 = exit su; never an obstacle   */
    int32_t n_peds;           /* number of pedestrians, 0..SF_MAX_PEDS; id =
                                 index in pos                                    */
    const int32_t *pos;       /* [n_peds] linear su index, distinct, on free
                                 non-exit su                                      */
    int32_t radius;           /* pedestrian field half-width R, 0..SF_MAX_RADIUS */
    double k, alpha;          /* pedestrian field law (paper example: 1, -0.5)   */
    double k_obs, alpha_obs;  /* obstacle field law                               */
    int32_t radius_obs;       /* obstacle field half-width; -1 = same as radius  */
    double w_dest;            /* weight of the destination field                  */
    uint64_t seed;            /* election key of the counter-based generator      */
    int64_t start_step;       /* tick index of the initial state (>= 0)           */
    /* The periodic workload of the paper's experiments (section 5): */
    int32_t periodic;         /* 1: both axes wrap (a torus): field windows and
                                 moves cross the edges; no obstacle or exit su
                                 may be set and width must be >= 64; 0: walls
                                 and exits as above                               */
    const uint8_t *heading;   /* [n_peds] per pedestrian: 0 = none, d = 1..8 the
                                 direction e_d of the direction list; a move e_m
                                 gets -w_heading * cos(angle(e_d, e_m)) added to
                                 its value (staying: 0).  NULL = no headings;
                                 copied                                          */
    double w_heading;         /* weight of the heading term                       */
    const uint8_t *walk_period; /* [n_peds] per pedestrian, >= 1: pedestrian i acts
                                 only on ticks t with (t + i) mod p_i = 0 and rests
                                 (stays, registers for nothing) on the others.
                                 NULL = every pedestrian acts every tick; copied */
    /* Pedestrians larger than one su (section 2; Table VI): */
    int32_t body_w, body_h;   /* body width and height in su, odd, 1..SF_MAX_BODY
                                 (0 reads as 1): pedestrian i covers the block
                                 centred on pos[i]; bodies lie in the grid (or
                                 wrap on a torus), cover no obstacle or exit and
                                 never overlap.  A move needs the whole shifted
                                 body free; a mover registers for the su its
                                 body enters and wins if its key is the
                                 smallest at all of them; a winner whose body
                                 reaches an exit leaves; the field radiates
                                 from the centre.  Scenes with bodies larger
                                 than 1 x 1 cannot join a batch.             */
} sf_scene_desc;

/* Running totals of a scene. */
typedef struct {
    int64_t step;      /* index of the next tick                                  */
    int64_t live;      /* pedestrians still in the scene                          */
    int64_t evacuated; /* pedestrians that left through an exit, in total        */
    int64_t ped_steps; /* sum over ticks run of the live count at the tick start */
    int64_t movers;    /* sum of pedestrians that registered for an su            */
    int64_t moved;     /* sum of pedestrians that won their election and moved    */
    int64_t tied;      /* sum of decisions whose two best FP32 values were within
                          1e-5 relative (near ties)                               */
    int64_t max_claimants; /* most pedestrians that registered for one su in one
                          tick, over all ticks run (section 3.1, s-2: at most 8
                          under v_max = 1)                                        */
} sf_stats_t;

/* Flags reported per pedestrian by sf_last_moves. */
#define SF_FLAG_MOVER 1u /* registered for a neighbour su (Algorithm 1, k-2)  */
#define SF_FLAG_WON 2u   /* won the election and moved (k-3, k-4)             */
#define SF_FLAG_TIED 4u  /* two best candidates within 1e-5 relative (FP32)   */

/* Kernels that sf_kernel_time can report. */
#define SF_KERNEL_SUPERPOSE 0 /* field write-back (k-5 role): P from positions  */
#define SF_KERNEL_DECIDE 1    /* decide + register (k-2, k-3 roles)             */
#define SF_KERNEL_COMMIT 2    /* move winners, evacuate (k-4)                    */
#define SF_KERNEL_COUNT 3

/* Create a scene: validate the descriptor, copy it to the device, build the
 * static fields (BFS destination field and obstacle field, fused to one FP32
 * array; zero on a periodic scene), bin the pedestrians and compute the field
 * of the initial positions.  `hip_stream` is a hipStream_t (NULL for the null
 * stream).  Blocks until the scene is ready.  Errors: SF_EINVAL (bad sizes,
 * pointers, radius, non-finite parameters, exit on an obstacle, no exit,
 * pedestrian out of range / on an obstacle or exit / duplicated, heading
 * above 8, walk period 0; periodic: an obstacle or exit su, width < 64, 2R+1
 * above a side),
 * SF_EUNREACHABLE (a free su cannot reach an exit), SF_ENOMEM, SF_EDEVICE.
 * On error *out is NULL. */
int sf_create_scene(const sf_scene_desc *desc, void *hip_stream, sf_scene **out);

/* Enqueue n_steps ticks (Algorithm 1 loop body, n_steps >= 0) on the scene's
 * stream and return without waiting.  After each tick the scene's field is
 * that of the new positions. */
int sf_step(sf_scene *s, int32_t n_steps);

/* Copy the current total field P (float32 [height*width], +inf on obstacle
 * su): the superposed field that k-5 writes back to the paper's shared field
 * store at the end of a tick (Algorithm 1; sections 2 and 3.1), summed as
 * Algorithms 2/3 and Eq. 1 sum it (any partition of the terms, the same
 * total).  dst_on_device = 1: dst is device memory and the copy is enqueued
 * on the scene's stream; 0: dst is host memory and the call blocks.  The
 * caller owns dst, which must hold height*width floats.  SF_EINVAL for a NULL
 * scene or dst; SF_EDEVICE if the copy fails. */
int sf_field(const sf_scene *s, float *dst, int dst_on_device);

/* Copy positions by pedestrian id (int32 [n_peds]: the centre su of section
 * 2's discrete model, -1 once the pedestrian has left through an opening, Fig.
 * 6 caption task 11) and, if `alive` is not NULL, alive flags (uint8 [n_peds],
 * host memory only).  Same dst_on_device convention as sf_field; the caller
 * owns both buffers.  SF_EINVAL for a NULL scene or pos, or alive flags asked
 * for on the device; SF_EDEVICE if a copy fails. */
int sf_positions(const sf_scene *s, int32_t *pos, uint8_t *alive, int dst_on_device);

/* Outcome of the last tick by pedestrian id (Algorithm 1: the su chosen by
 * k-2, the election of k-3, the move of k-4): target su (int32 [n_peds]; own
 * su when staying, -1 when already evacuated before that tick) and SF_FLAG_*
 * bits (uint8 [n_peds]).  Either pointer may be NULL.  Same dst_on_device
 * convention as sf_field.  Before the first tick all entries are zero. */
int sf_last_moves(const sf_scene *s, int32_t *target, uint8_t *flags, int dst_on_device);

/* Copy the static fields (section 2: the openings' attractive and the
 * obstacles' repulsive field): S = w_dest*D + O (float64 [height*width],
 * +inf on obstacles) and D (int32 [height*width], -1 on obstacles).  Either
 * pointer may be NULL.  Same dst_on_device convention as sf_field. */
int sf_static_field(const sf_scene *s, double *S, int32_t *D, int dst_on_device);

/* Replace the pedestrian state (checkpoint resume): host positions by id
 * (int32 [n_peds], -1 = evacuated; live ones distinct, on free non-exit su,
 * as section 2 requires) and the index of the next tick t of Algorithm 1's
 * loop.  Counters are reset as at creation with the evacuated count set to
 * the number of -1 entries.  Blocks.  SF_EINVAL on a bad state. */
int sf_set_state(sf_scene *s, const int32_t *pos, int64_t step);

/* Copy the running totals of the ticks run (Algorithm 1's loop: registrations
 * of k-2, elections of k-3 with section 3.1's s-2 bound of 8 registrants per
 * su, moves of k-4, departures through openings).  Blocks until the scene's
 * queued work is done.  SF_EINVAL for a NULL argument; SF_EDEVICE if the copy
 * fails. */
int sf_stats(const sf_scene *s, sf_stats_t *out);

/* Block until all work enqueued for the scene has finished (the host side of
 * the paper's command-queue synchronisation, section 4).  SF_EINVAL for a
 * NULL scene; SF_EDEVICE if the stream reports an error. */
int sf_sync(const sf_scene *s);

/* Field update mode.  refresh_ticks <= 1 (default 0): the field is
 * superposed from all pedestrians every tick.  refresh_ticks = K >= 2: the
 * incremental update of Algorithm 1 (k-4 buffers the field changes of the
 * pedestrians that moved, k-5 writes them back): between full superpositions,
 * a tick adds the stamps at the su its winners entered and subtracts those at
 * the su they left, into an exact FP64 pedestrian field the scene keeps (8 B
 * per su), and every K-th tick the field is superposed in full again.  The
 * sums are exact, so every updated field is the full superposition of the
 * same positions bit for bit, whatever K.  The update is one launch of the
 * superposition kernel with the su entered and the su left as two source
 * sets.  Blocks.  SF_EINVAL for a negative value or a scene that belongs to a
 * batch; SF_ENOMEM if the FP64 field cannot be allocated. */
int sf_set_field_update(sf_scene *s, int32_t refresh_ticks);

/* The paper's own field path instead of the exact gather (section 3.1, s-1:
 * each su keeps its strengths in 8 sects, the "3-D image", and the strength a
 * source at o puts at su c lands in the sect of the offset c - o; the number
 * of window offsets per sect is the strength fan-out SF; Algorithm 3 with
 * Eq. 1: an su's 8*SF fan-out terms, zero padded to a multiple of K, are
 * summed in K blocks of m consecutive terms, each into one FP32 slot, and the
 * K slots are summed).  Readings: sect = floor(angle(c - o) / 45 degrees),
 * the angle from +x toward +y in [0, 360) (SF = R(R+1)/2; the paper's 7x7
 * field has 6); terms sect by sect, row-major within a sect; block j = terms
 * j*m .. j*m + m - 1; all sums FP32 in that order; P = fl32(S + Phi32).
 * K = 2, 4, 8 or 16 selects the path; K = 0 returns to the exact gather.
 * keep_image = 1 also keeps the 8 sect planes (sf_sect_image; 32 B per su).
 * With sf_set_field_update(K' >= 2) the ticks between full fields add the
 * FP32 sums of the strengths at the su entered (+) and left (-) to the kept
 * FP32 field and image: the incremental k-4/k-5 of Algorithm 1, whose FP32
 * rounding drifts until the next full field.  The field is recomputed at
 * once; blocks.  SF_EINVAL for another K or a scene in a batch (batches keep
 * the gather); SF_ENOMEM if the FP32 field or image cannot be allocated. */
int sf_set_field_sect(sf_scene *s, int32_t K, int32_t keep_image);

/* The 8 sect planes of the sect path (8 x height x width floats, plane s =
 * sect s of every su; the FP32 sums of that sect's terms), as kept by
 * sf_set_field_sect with keep_image = 1; copy semantics as sf_field.
 * SF_EINVAL when the scene keeps no image. */
int sf_sect_image(const sf_scene *s, float *dst, int dst_on_device);

/* Superpose the field of the current positions again, n_times times (no
 * tick; positions, counters and step index unchanged): k-5's write-back of
 * Algorithm 1 alone.  The result is the field sf_step leaves after a tick, bit
 * for bit, so repeated calls change nothing; under the incremental update
 * (sf_set_field_update) it starts a new refresh period.  Enqueued on the
 * scene's stream (timed as SF_KERNEL_SUPERPOSE); does not block.  SF_EINVAL
 * for a negative count or a scene that belongs to a batch. */
int sf_refresh_field(sf_scene *s, int32_t n_times);

/* Superposition without a scene: k-5's field write-back of Algorithm 1 for a
 * caller's set of pedestrians (Algorithms 2 and 3 with Eq. 1: the field of an
 * su is the sum of the strengths that the sources in its window put there,
 * in any order).  For every su c of a width x height grid
 *     P[c] = fl32(S[c] + sum over j < n with 0 <= pos[j] < width*height of
 *                 phi(c - pos[j])),
 * phi(d) = fl32(k*|d|_2^alpha) for 0 < |d|_inf <= radius, 0 elsewhere (on a
 * torus, periodic = 1, the nearest image of each source), the sum formed
 * exactly in FP64 (the law must pass the check of sf_create_scene) and
 * rounded once.
 *   S    device, double[width*height]: the static field (+inf on obstacle su
 *        gives P = +inf there); read only.
 *   pos  device, int32[n]: linear su indices; entries outside
 *        0..width*height-1 (-1 for an absent pedestrian) are skipped, and a
 *        repeated su counts once (the sources are the set of occupied su).
 *   P    device, float[width*height]: written.
 * The pointers belong to the caller and to the device current at the call.
 * The work is enqueued on hip_stream (NULL = the null stream) and the call
 * returns before it completes; its scratch (an occupancy bitmap of width*height
 * bits and the stamp table, at most 160 KiB) is allocated and freed in stream
 * order (hipMallocAsync / hipFreeAsync).  The same grid limits as a scene:
 * SF_EINVAL for sizes, radius (0..SF_MAX_RADIUS; a torus needs width >= 64
 * and 2*radius+1 <= both sides), a law refused by the exactness check,
 * periodic not 0/1, n < 0, or a NULL S, P (or pos with n > 0); SF_ENOMEM when
 * the scratch cannot be allocated; SF_EDEVICE for a HIP error. */
int sf_superpose(int32_t width, int32_t height, int32_t periodic, int32_t radius, double k,
                 double alpha, const double *S, const int32_t *pos, int32_t n, float *P,
                 void *hip_stream);

/* sf_superpose for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, the same kernels and the same result bit for bit, with no
 * hipMalloc, hipFree or other allocating call.  Its scratch (bitmap and stamp)
 * is a static device array of 8.25 MiB that each device the library runs on
 * holds until the process ends; grids whose bitmap needs more than 2^20 words
 * (ceil(width/64)*height; 8192 x 8192 is the largest square) are refused
 * with SF_EINVAL.  Every
 * call on one device shares that array and leaves its last contents there
 * (the call clears what it needs): calls that overlap on one device, on
 * different streams or threads, race and give undefined fields; calls on one
 * stream are ordered.  Errors as for sf_superpose, without SF_ENOMEM. */
int sf_superpose_noalloc(int32_t width, int32_t height, int32_t periodic, int32_t radius,
                         double k, double alpha, const double *S, const int32_t *pos, int32_t n,
                         float *P, void *hip_stream);

/* Per-kernel timing of the tick's kernels (the per-job time profile of the
 * paper's Fig. 7): while enabled, every launch of the kernels listed above
 * records a start/stop HIP event pair as part of its own dispatch (the
 * kernel's execution interval, no extra stream packets).  enable = 1 starts a
 * fresh measurement, 0 stops recording.  sf_kernel_time blocks, then reports
 * the summed duration in milliseconds and the number of launches measured for
 * one SF_KERNEL_* id (SF_EINVAL for a NULL argument or an unknown id). */
int sf_set_timing(sf_scene *s, int enable);
int sf_kernel_time(const sf_scene *s, int kernel, double *total_ms, int64_t *launches);

/* Release the scene and all its device memory (NULL is ignored): the end of
 * Algorithm 1's simulation period.  Waits for the scene's work first.  A batch
 * that still holds the scene can no longer step (sf_batch_step then fails
 * with SF_EINVAL). */
void sf_destroy_scene(sf_scene *s);

/* ---- batches ---------------------------------------------------------------
 * Not in the paper, whose tick runs one scene at a time: a batch advances many
 * scenes of different grid size, crowd and radius together.  Each tick is one
 * decide, one commit and one field launch that together cover every member
 * scene, and runs of ticks are replayed from captured HIP graphs.  Every
 * member evolves exactly as under sf_step alone: the kernels are the same,
 * per scene, and the field's summation order does not depend on the launch.
 * (Scenes are split into at most SF_MAX_GROUPS groups by radius, each with its
 * own three launches per tick; see sf_batch_tiling.)
 *
 * While a scene belongs to a batch its work runs on the batch's stream:
 * sf_field, sf_positions, sf_last_moves, sf_static_field, sf_stats and sf_sync
 * on the scene are ordered after the batch's enqueued ticks, while sf_step and
 * sf_set_state on it fail with SF_EINVAL.  A scene belongs to at most one batch
 * at a time, and scenes in the incremental field update mode cannot join one.  Destroy a batch before its scenes; if a member scene is destroyed
 * first, later sf_batch_step calls on that batch fail with SF_EINVAL. */
typedef struct sf_batch sf_batch; /* opaque, library-owned */

/* Launch shape and schedule of one group of a batch (a zero field = library
 * default). */
typedef struct {
    int32_t tw, hl, vec, nw;   /* field kernel: strip width in su, rows per lane,
                                  stamp entries per LDS read (2: paired loads;
                                  4: 16-byte loads, integer stamps and hl 4
                                  or 8 only), waves per workgroup; one of the
                                  compiled shapes, or all four zero (vec 0
                                  reads as 2)                                  */
    int32_t list_cap;          /* field kernel: source-list entries in LDS      */
    int32_t blocks_per_cu;     /* field kernel: workgroups per compute unit     */
    int32_t items_per_block;   /* field kernel: work items (runs of strips of
                                  one scene) dealt to each workgroup per tick  */
} sf_group_tiling;

/* A batch splits its scenes into up to SF_MAX_GROUPS groups by field radius:
 * group g holds the scenes with split_radius[g-1] < radius <= split_radius[g]
 * (group 0 from radius 0, the last group up to the largest radius).  Each
 * group has its own launches and tiling (small and large stamps favour
 * different tile shapes and LDS budgets), and the groups' ticks run as
 * independent streams of work that the GPU overlaps. */
#define SF_MAX_GROUPS 4
typedef struct {
    int32_t groups;            /* 0 = default: one group per distinct radius when
                                  there are at most SF_MAX_GROUPS of them, else
                                  SF_MAX_GROUPS groups of about equal estimated
                                  field work; 1..SF_MAX_GROUPS = that many
                                  (each must be non-empty)                      */
    int32_t split_radius[SF_MAX_GROUPS - 1];
                               /* upper radius of groups 0..groups-2, strictly
                                  increasing; all zero = chosen as for the
                                  default (two groups: split at radius 8)       */
    sf_group_tiling group[SF_MAX_GROUPS];
} sf_batch_tiling;

/* Group n_scenes (>= 1, distinct, none in another batch, all on the current
 * device) into a batch whose ticks are enqueued on `hip_stream`.  `tiling`
 * may be NULL (defaults).  Waits for the scenes' queued work.  The scenes
 * stay owned by the caller.  Errors: SF_EINVAL (bad list or tiling that does
 * not fit the largest radius), SF_ENOMEM, SF_EDEVICE. */
int sf_batch_create(sf_scene *const *scenes, int32_t n_scenes, const sf_batch_tiling *tiling,
                    void *hip_stream, sf_batch **out);

/* Autotuner: for each group, times the field launch of every compiled shape
 * and a few schedules on the batch's current state (`reps` launches each,
 * median kept), adopts the fastest and, if `chosen` is not NULL, reports it.  The
 * scenes' state is unchanged (the field is recomputed, bit for bit).
 * Blocks. */
int sf_batch_tune(sf_batch *b, int32_t reps, sf_batch_tiling *chosen);

/* The tiling in use (defaults filled in). */
int sf_batch_get_tiling(const sf_batch *b, sf_batch_tiling *out);

/* Enqueue n_steps (>= 0) ticks of every member scene and return without
 * waiting.  Runs of two or more ticks replay graphs of up to 8 ticks,
 * captured on first use; a single tick is launched directly. */
int sf_batch_step(sf_batch *b, int32_t n_steps);

/* Superpose the field of every member scene again, n_times times (no tick;
 * positions, counters and step index unchanged; the fields keep their bits):
 * the field launch of each group in turn, back to back on the batch's stream
 * (k-5's write-back of Algorithm 1 for all members).  For timing the batched
 * field.  Does not block.  SF_EINVAL for a negative count or a batch whose
 * member was destroyed. */
int sf_batch_refresh_field(sf_batch *b, int32_t n_times);

/* Running totals of every member scene (out[n_scenes], in the order given to
 * sf_batch_create), read with one launch and one copy.  Blocks until the
 * batch's queued work is done. */
int sf_batch_stats(const sf_batch *b, sf_stats_t *out);

/* Block until all work enqueued on the batch has finished. */
int sf_batch_sync(const sf_batch *b);

/* Release the batch (NULL is ignored) after its work; the member scenes go
 * back to their own streams. */
void sf_batch_destroy(sf_batch *b);

/* Number of HIP devices visible to the library's HIP runtime (0 without one
 * or when the runtime cannot start; never fails).  A process must hold one
 * HIP runtime: a host program that carries its own (a framework's) loads it
 * before this library, so that the library binds to it. */
int sf_device_count(void);

/* Message of the last failure on the calling thread ("" if none). */
const char *sf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SF_H */
