/* spasm.h -- C ABI of the MI355X (gfx950) SPaSM particle engine.
 *
 * SPaSM (Chen, Iyer, Kingston, "Differentiable Particle Optimization for Fast
 * Sequential Manipulation", arXiv 2510.07674) solves pick-and-place for a given action
 * skeleton in two stages: stage 1 samples and optimises block placements (Alg. 1),
 * stage 2 lifts the surviving placements to joint-space trajectories and descends the
 * whole trajectory together with the placements (Sec. III-B, Appendix B).  This library
 * runs both stages as HIP kernels on the device; the caller owns every device buffer.
 *
 * Conventions shared by every entry point:
 *   - All d_* arguments are device pointers (hipMalloc'd or torch tensors'
 *     data_ptr()), contiguous, row-major, float32 unless stated.  Host pointers are
 *     never retained past the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Device
 *     entry points only enqueue work on it and return; spasm_solve synchronises it.
 *   - A problem may be used from one stream at a time.  Calls on different problems are
 *     independent.
 *   - Return value: SPASM_OK or a negative status; spasm_last_error() returns a
 *     thread-local message describing the last failure.  Invalid sizes, NULL buffers,
 *     non-finite descriptions and unsupported shapes are rejected before any launch.
 *     An infeasible problem is not an error: spasm_solve reports success = 0.
 *
 * State layouts (per particle p):
 *   stage-1 placement  x    [N][B][3]      block x, y, yaw (z fixed at its slot)
 *   stage-2 trajectory q    [P][2B][W][7]  segment s = 2b: transit to block b;
 *                                          s = 2b+1: transfer of block b; the last
 *                                          waypoint of s and the first of s+1 are copies
 *                                          of one configuration
 *   stage-2 placement  pose [P][B][4]      block x, y, z, yaw
 */
#ifndef SPASM_H
#define SPASM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPASM_OK 0
#define SPASM_EINVAL (-1)      /* bad argument: size, NULL, non-finite value */
#define SPASM_ENOMEM (-2)      /* device allocation failed (problem_create only) */
#define SPASM_EHIP (-3)        /* a HIP runtime call failed */
#define SPASM_EUNSUPPORTED (-4) /* shape outside what the kernels support */
#define SPASM_EBUSY (-5)       /* serving: no free slot or HBM budget */

#define SPASM_STAGE_PLACE 1
#define SPASM_STAGE_TRAJ 2
#define SPASM_PHASE_LIN 0      /* residuals as they are (Sec. III-A, linear cost) */
#define SPASM_PHASE_QUAD 1     /* squared residuals (quadratic refinement) */
#define SPASM_MODE_TOWER 0     /* block b goes to tower slot b, centre height (b + 1/2) h */
#define SPASM_MODE_FIXED 1     /* block b goes to goal[b] */
#define SPASM_MODE_PACK 2      /* polyomino pieces packed into the region (stage 1 only) */
#define SPASM_MODE_P2P 3       /* one motion from q_home to p2p_goal (trajectory only) */

typedef struct spasm_problem_s *spasm_problem;

/* Serial chain: 7 revolute joints, classic DH A_k = Rz(q_k) Tz(d_k) Tx(a_k) Rx(alpha_k),
 * base frame = world (z up), end effector T_E = T_7 Tz(tool_d). */
typedef struct {
    double dh[7][3];     /* a, d, alpha */
    double lo[7], hi[7]; /* joint limits */
    double tool_d;
    double q_home[7];    /* start of the first segment when seeding trajectories */
} spasm_chain_desc;

/* Blocks and action skeleton: block b is picked from block_init[b] and placed either on
 * the tower (slot b) or at goal[b]; blocks are moved in index order.
 * Packing (SPASM_MODE_PACK, the Tetris problem of Sec. IV and Appendix A): block b is a
 * piece made of pack_cells[b] square cells of edge block_edge centred at pack_off[b][k]
 * in the piece frame; the pieces are packed into the region, whose four sides are the
 * walls.  Packing problems support the stage-1 entry points only (sample, placement
 * cost, stage-1 optimize, selection, order, place_round); the stage-2 entry points
 * return SPASM_EUNSUPPORTED for them.
 * Point to point (SPASM_MODE_P2P, the motion-planning use of Sec. IV): one motion from
 * chain->q_home to p2p_goal among the obstacles, both within the joint limits; n_blocks
 * must be 1 (a placeholder, block_init may be NULL).  The trajectory has one segment,
 * q [P][1][W][7], whose first and last waypoints are pinned; its cost is the stage-2
 * cost of that segment without blocks (w_arm C_arm + w_lim C_lim + w_smooth C_smooth).
 * The stage-2 entry points take d_pose / d_gpose = NULL (no pose variables);
 * spasm_traj_init ignores d_qgrasp, d_qplace and d_pose; spasm_solve and
 * spasm_solve_ttfs take N1 = 0 and skip the lift; the IK entry points and the server
 * return SPASM_EUNSUPPORTED. */
typedef struct {
    int32_t n_blocks;         /* B >= 1 */
    int32_t mode;             /* SPASM_MODE_TOWER, SPASM_MODE_FIXED or SPASM_MODE_PACK */
    double block_edge;        /* h: cube edge */
    double block_margin;      /* block collision spheres have radius h/4 - margin */
    const double *block_init; /* host [B][4] x, y, z, yaw */
    const double *goal;       /* host [B][4] (SPASM_MODE_FIXED), ignored for towers */
    double grasp[3][4];       /* G: block frame -> end-effector frame, [R | t] */
    double region[4];         /* placement bounding box x_lo, x_hi, y_lo, y_hi */
    const int32_t *pack_cells; /* host [B] cells per piece, 1..8 (SPASM_MODE_PACK), else NULL */
    const double *pack_off;    /* host [B][8][2] cell centres in the piece frame (rows k >=
                                * pack_cells[b] ignored); cells of one piece must not overlap */
    int32_t sample_yaw_steps;  /* stage-1 yaw samples: 0 = uniform in [-pi, pi); n in 1..64 =
                                * the n directions -pi + 2 pi j / n */
    const double *p2p_goal;    /* host [7] goal configuration (SPASM_MODE_P2P), else NULL */
} spasm_skeleton_desc;

/* Weights and schedules.  Stage 1 (Alg. 1): k_lin1 linear steps with
 * eta_k = eta1 (1 - k / k_lin1), then k_quad1 quadratic steps at alpha1.  Stage 2: Adam
 * (beta1, beta2, adam_eps, bias-corrected) under the same schedule shape over K steps
 * with k_lin2 = round(lin_frac2 K), eta2, alpha2. */
typedef struct {
    double w[9];   /* stable, height, coll, start, tie, arm, block, lim, smooth */
    int32_t k_lin1, k_quad1;
    double eta1, alpha1;
    double lin_frac2, eta2, alpha2, beta1, beta2, adam_eps;
    int32_t ik_iters;
    int32_t ik_restarts;  /* IK starts per (particle, block) in the lift, 1..8 */
    int32_t mid_candidates;  /* intermediate-waypoint draws per segment in the seeding, 1..8 */
    double ik_lambda, ik_noise, mid_noise;
    double sat_eps;   /* a particle satisfies the constraints when its violation < sat_eps */
    int32_t retries;  /* stage-1 resampling rounds when nothing satisfies */
    /* Augmented-Lagrangian outer loop of stage 2 (Sec. III-B), off when al_every = 0: each
     * block's grasp residual e (position, z axis: 6 components) and tie residual (position,
     * x axis, z axis: 9) get multipliers lambda, the cost gains lambda . e, and after the
     * evaluation of every al_every-th iteration lambda += al_rho * 2 w e (w_start, w_tie).
     * Multipliers start at zero in spasm_solve / spasm_solve_ttfs; the server takes
     * al_every = 0 only. */
    int32_t al_every;
    double al_rho;
} spasm_params;

typedef struct {
    int32_t N1;    /* stage-1 samples; 0 = fixed goals, no stage 1 */
    int32_t M;     /* particles kept after stage 1 = stage-2 particles */
    int32_t W;     /* waypoints per segment: 4, 8, 16, 32 or 64 */
    int32_t K;     /* stage-2 iterations */
    uint64_t seed;
} spasm_solve_config;

typedef struct {
    int32_t success;     /* 1 if the best particle's violation < sat_eps */
    int32_t n_sat;       /* satisfying stage-2 particles */
    int32_t stage1_sat;  /* satisfying stage-1 particles in the committed round (-1: none run) */
    int32_t rounds;      /* stage-1 rounds run */
    int32_t best;        /* index of the returned particle */
    float viol, cost;    /* of the returned particle (quadratic phase) */
    float length;        /* configuration-space path length sum |q_{w+1} - q_w| (rad) */
    float stage1_ms, stage2_ms, total_ms;  /* device time (HIP events) */
    float opt_ms;        /* the fused stage-2 descent launch alone */
} spasm_result;

/* --- problem -------------------------------------------------------------------------
 * Copies the description to the current device (about 1-4 KB).  Spheres: n_sph of them,
 * sph_link[i] in 1..7 non-decreasing, sph_c [n_sph][3] centres in the link frame,
 * sph_r [n_sph] radii.  Obstacles: n_obs axis-aligned boxes [n_obs][6] centre and half
 * extents (Sec. III: robot and objects as spheres, penetration penalties).  The problem
 * owns its device copy until spasm_problem_destroy. */
int spasm_problem_create(const spasm_chain_desc *chain, int32_t n_sph, const int32_t *sph_link,
                         const double *sph_c, const double *sph_r, int32_t n_obs,
                         const double *boxes, const spasm_skeleton_desc *skel,
                         const spasm_params *prm, spasm_problem *out);
void spasm_problem_destroy(spasm_problem prob);
int spasm_problem_blocks(spasm_problem prob);

/* --- stage 1 --------------------------------------------------------------------------
 * Alg. 1 SampleUniform: N placements, x and y uniform over the region shrunk by h/2, yaw
 * uniform in [-pi, pi) (or, with sample_yaw_steps = n > 0, -pi + (2 pi / n) floor(n u)).
 * Philox4x64-10 with key (seed, 0) and counter (particle, block, round, 1); uniforms are
 * the top 24 bits.  d_x: [N][B][3]. */
int spasm_sample(spasm_problem prob, int32_t N, uint64_t seed, int32_t round, float *d_x,
                 void *stream);

/* --- costs ----------------------------------------------------------------------------
 * Cost, violation and gradient of a batch (Appendix B).
 * stage SPASM_STAGE_PLACE: d_x [P][B][3] placements; C_placement with z at the slot
 *   heights; d_gx [P][B][3]; W and d_pose unused.  Packing problems (Appendix A): the sum
 *   over cell pairs of different pieces of the squares' penetration depth (separating
 *   axis theorem) plus the sum over cells of the depth past each wall, weighted by
 *   w_coll and passed through the phase's penalty (identity or square).
 * stage SPASM_STAGE_TRAJ: d_x = q [P][2B][W][7], d_pose [P][B][4];
 *   C_trajopt = C_placement(pose) + w_start C_start + w_tie C_tie + w_arm (C_arm + arm vs
 *   blocks) + w_block C_block + w_lim C_lim + w_smooth C_smooth.  d_gx [P][2B][W][7] is the
 *   gradient of every waypoint copy separately; d_gpose [P][B][4].
 * d_cost [P], d_viol [P] (largest unsquared, unweighted residual).  d_gx / d_gpose may be
 * NULL to compute costs only. */
int spasm_cost_grad(spasm_problem prob, int32_t stage, int32_t phase, int32_t P, int32_t W,
                    const float *d_x, const float *d_pose, float *d_cost, float *d_viol,
                    float *d_gx, float *d_gpose, void *stream);

/* Stage-2 cost and gradient with the augmented-Lagrangian multiplier terms (see
 * spasm_params.al_every): d_lambda [P][B][15] (grasp residual components 0..5, tie
 * residual 6..14 per block), read only; otherwise as spasm_cost_grad at stage 2. */
int spasm_cost_grad_al(spasm_problem prob, int32_t phase, int32_t P, int32_t W, const float *d_q,
                       const float *d_pose, const float *d_lambda, float *d_cost, float *d_viol,
                       float *d_gq, float *d_gpose, void *stream);

/* Adjoint of the stage-2 cost for reverse-mode differentiation: given d_gout [P]
 * (dL/dcost per particle) writes d_gq = gout * dcost/dq [P][2B][W][7] and
 * d_gpose = gout * dcost/dpose [P][B][4]. */
int spasm_cost_adjoint(spasm_problem prob, int32_t phase, int32_t P, int32_t W, const float *d_q,
                       const float *d_pose, const float *d_gout, float *d_gq, float *d_gpose,
                       void *stream);

/* --- updates --------------------------------------------------------------------------
 * Runs global schedule steps k_begin .. k_end-1 (1-based) in ONE launch, each a fused
 * cost + gradient + update per particle with the state held on chip.
 * stage 1 (Alg. 1 lines 5-14): gradient descent on d_x [P][B][3], x and y clamped into
 *   the region shrunk by h/2; steps 1..k_lin1 linear, then quadratic; d_pose, d_opt unused.
 * stage 2 (Sec. III-B): Adam on d_x = q [P][2B][W][7] and, for towers, d_pose [P][B][4];
 *   K_total sets k_lin2; boundary copies get the sum of their gradients;
 *   d_opt holds the Adam moments [P][(2B*W*7 + 4B) * 2] floats (m then v per particle),
 *   and, when al_every > 0, each particle's 15B multipliers after its moments (row of
 *   (2B*W*7 + 4B) * 2 + 15B floats); read at entry and written back at exit; zero it
 *   before step 1.
 * d_cost / d_viol (nullable, [P]) receive the quadratic-phase cost and violation of the
 * final state. */
int spasm_optimize(spasm_problem prob, int32_t stage, int32_t P, int32_t W, float *d_x,
                   float *d_pose, float *d_opt, int32_t k_begin, int32_t k_end, int32_t K_total,
                   float *d_cost, float *d_viol, void *stream);

/* --- selection ------------------------------------------------------------------------
 * Alg. 1 ArgSort[:M]: indices of the M smallest keys, ascending, equal keys in index
 * order.  1 <= M <= N <= 16384.  d_key [N], d_idx [M] int32.  Computed by rank: (key,
 * index) pairs are unique, so each one's sorted position is the count of pairs below it,
 * counted by up to 256 workgroups at once. */
int spasm_select_topm(int32_t N, const float *d_key, int32_t M, int32_t *d_idx, void *stream);

/* The same selection for up to 2^20 keys (M <= 8192 when N > 16384): a radix select
 * (three counting passes over the ordered cost bits find the M-th smallest cost T; the
 * keys below T and the first keys equal to T in index order are collected) followed by
 * the rank selection of those M keys, so the result equals the stable sort's first M.
 * d_work: spasm_select_topm_workspace(N, M) bytes, 256-byte aligned (0 for N <= 16384;
 * d_work may then be NULL). */
size_t spasm_select_topm_workspace(int32_t N, int32_t M);
int spasm_select_topm_large(int32_t N, const float *d_key, int32_t M, int32_t *d_idx, void *d_work,
                            size_t work_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the selection of
 * spasm_select_topm_large without a workspace.  Its scratch (the select state, histogram,
 * per-range counts and survivors) is one static device array per GPU of
 * spasm_select_topm_static_bytes() bytes (about 74 KB, held until the process ends),
 * enough for every supported shape: 1 <= M <= N <= 2^20, M <= 8192 when N > 16384; larger
 * sizes return SPASM_EUNSUPPORTED.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine); each call resets the scratch it reads.  Calls that overlap
 * on one GPU (concurrent streams or threads) share that array and race: serialise them. */
size_t spasm_select_topm_static_bytes(void);
int spasm_select_topm_static(int32_t N, const float *d_key, int32_t M, int32_t *d_idx, void *stream);

/* Alg. 1 GetSatisfyingParticles + re-evaluated ArgSort: order of all n particles with the
 * satisfying ones (viol < eps) first, each group by cost then index; d_nsat [1] int32
 * receives the number of satisfying particles.  n <= 16384. */
int spasm_order(int32_t n, const float *d_cost, const float *d_viol, float eps, int32_t *d_order,
                int32_t *d_nsat, void *stream);

/* --- sampled placements (Alg. 1 lines 1-4) ---------------------------------------------------
 * Draws N placements (round `round` of the sample stream, as spasm_sample), scores each
 * with the linear-phase placement cost (Alg. 1 Cost) and keeps the M lowest-cost samples
 * (ArgSort[:M]: ascending cost, equal costs in sample order; N up to 2^20 as in
 * spasm_select_topm_large).  d_place [M][B][3] the kept samples in that order, d_cost /
 * d_viol [M] (nullable) their linear-phase cost and violation.  d_work:
 * spasm_sample_placements_workspace(prob, N, M) bytes, 256-byte aligned (0 returned for an
 * unsupported shape). */
size_t spasm_sample_placements_workspace(spasm_problem prob, int32_t N, int32_t M);
int spasm_sample_placements(spasm_problem prob, int32_t N, int32_t M, uint64_t seed, int32_t round,
                            void *d_work, size_t work_bytes, float *d_place, float *d_cost, float *d_viol,
                            void *stream);

/* --- whole stage 1 (Alg. 1 lines 1-23) -------------------------------------------------------
 * The stage 1 that spasm_solve runs: rounds r = 0, 1, ... of sampling N placements, the
 * linear score, the M best, the k_lin1 + k_quad1 descent and the satisfying-first order,
 * until a round has a satisfying particle or 1 + retries rounds have run (the last round's
 * particles are then kept anyway); the decision is taken on the device, later rounds'
 * kernels exit at once.  Towers and packing problems; 1 <= M <= N <= 16384.
 * d_pose [M][B][4]: the committed round's placements in satisfying-first order, as stage-2
 * placement variables (x, y, slot-height z, yaw); d_cost / d_viol [M] (nullable): their
 * quadratic-phase cost and violation; d_info [2] int32: satisfying particles of the
 * committed round, rounds run.  d_work: spasm_stage1_workspace(prob, N, M) bytes, 256-byte
 * aligned (0 returned for an unsupported problem or shape). */
size_t spasm_stage1_workspace(spasm_problem prob, int32_t N, int32_t M);
int spasm_stage1(spasm_problem prob, int32_t N, int32_t M, uint64_t seed, void *d_work, size_t work_bytes,
                 float *d_pose, float *d_cost, float *d_viol, int32_t *d_info, void *stream);

/* --- placement only (Alg. 1, one round) ---------------------------------------------------
 * Stage 1 without trajectory optimisation: sample N placements (round `round` of the
 * sample stream), score them (linear phase), keep the M best (N up to 2^20 as in
 * spasm_select_topm_large), run the k_lin1 + k_quad1 descent on them, and write them in
 * satisfying-first order: d_x [M][B][3] (x, y, yaw), d_cost / d_viol [M] (nullable,
 * quadratic phase), d_nsat [1] the number of satisfying placements.  d_work:
 * spasm_place_workspace(prob, N, M) bytes, 256-byte aligned.  Callers that want the time
 * to a first feasible placement repeat rounds until *d_nsat > 0. */
size_t spasm_place_workspace(spasm_problem prob, int32_t N, int32_t M);
int spasm_place_round(spasm_problem prob, int32_t N, int32_t M, uint64_t seed, int32_t round, void *d_work,
                      size_t work_bytes, float *d_x, float *d_cost, float *d_viol, int32_t *d_nsat,
                      void *stream);

/* --- lift and seeding (Sec. III-B) -----------------------------------------------------
 * Damped least squares IK on the block frame T_E G^-1 (the paper allows any parallel
 * IK): dq = J^T (J J^T + lambda^2 I)^-1 e, clamped to the limits.
 * spasm_ik_iterate: n independent solves, in place on d_q [n][7], kind 0 = grasp (block
 *   origin to target xyz, block z axis up, yaw free), kind 1 = place (x, y, z, yaw);
 *   d_target [n][4].
 * spasm_ik_lift: per particle and block, ik_restarts multi-start solves.  Grasp at
 *   block_init[b]: start 0 at q_home + ik_noise U[-1,1]^7 (counter (particle, 2b + chunk,
 *   0, 2)), start r >= 1 uniform over the limits (counter (particle, 2b + chunk, r, 2)).
 *   Place at d_pose[p][b]: start 0 from the chosen grasp solution, start r >= 1 uniform
 *   (counter (particle, 2B + 2b + chunk, r, 2)).  Among the starts whose final error |e|
 *   (position and orientation error of the iteration) is below 1e-4 each solve keeps the
 *   one with the smallest clutter score (see spasm_traj_init; the first on ties); when
 *   none converged, the start with the smallest error (the first on ties).
 *   d_qgrasp, d_qplace [P][B][7]. */
int spasm_ik_iterate(spasm_problem prob, int32_t kind, int32_t n, const float *d_target, float *d_q,
                     int32_t iters, void *stream);
int spasm_ik_lift(spasm_problem prob, int32_t P, const float *d_pose, uint64_t seed, int32_t iters,
                  float *d_qgrasp, float *d_qplace, void *stream);

/* Straight-line seeds through one intermediate waypoint per segment, at index (W-1)/2;
 * the first segment starts at q_home.  The intermediate waypoint is the best of
 * mid_candidates draws c of the segment ends' midpoint plus mid_noise U[-1,1]^7 (counter
 * (particle, 2s + chunk, c, 3)), clamped to the limits: the draw whose seed path has the
 * smallest clutter score (below) summed at the intermediate waypoint and at the two
 * points halfway to the ends (the first on ties).  d_pose [P][B][4]: the placements.
 * d_q [P][2B][W][7].
 * Clutter score of q for block b (also used by the lift): the sum over robot spheres of
 * max(0, r - sdf) against every box and every block visible as in the stage-2 cost --
 * blocks below b at their placements, above b at their initial poses, block b at its
 * placement for a place configuration, at its initial pose inside its transit, not at
 * the grasp nor while held. */
int spasm_traj_init(spasm_problem prob, int32_t P, int32_t W, const float *d_qgrasp,
                    const float *d_qplace, const float *d_pose, uint64_t seed, float *d_q, void *stream);

/* --- whole method ------------------------------------------------------------------------
 * Stage 1 (cfg->N1 > 0): sample N1, score (linear phase), keep the best M, descend,
 * order satisfying first; resample up to `retries` more rounds while none satisfies
 * (decided on the device).  Fixed goals (N1 = 0): every particle starts at the goals.
 * Then lift, seed, K Adam steps, final quadratic-phase evaluation and the best particle.
 * When the particles need more waves than the device holds at once, they are ranked by
 * one cost evaluation of the seeded state and launched costliest first; each particle's
 * result does not depend on that order.
 * d_work: device workspace of spasm_solve_workspace() bytes (256-byte aligned).
 * d_best_q [2B][W][7] and d_best_pose [B][4] receive the returned particle; *out the
 * summary.  Synchronises the stream once at the end. */
size_t spasm_solve_workspace(spasm_problem prob, const spasm_solve_config *cfg);
int spasm_solve(spasm_problem prob, const spasm_solve_config *cfg, void *d_work, size_t work_bytes,
                float *d_best_q, float *d_best_pose, spasm_result *out, void *stream);

/* Device memory one spasm_solve of this configuration occupies, in bytes: its workspace
 * plus the d_best_q and d_best_pose outputs, each rounded up to 256 bytes (0 for an invalid
 * configuration).  The stage-2 Adam moments live in on-chip memory during the fused
 * launch and take no device memory; a served request also keeps them between steps (see
 * spasm_server_footprint). */
size_t spasm_solve_footprint(spasm_problem prob, const spasm_solve_config *cfg);

/* Time to first solution (the paper's solve-time measure, Sec. IV: time until a first
 * solution, at most 30,000 optimisation steps): attempts of the whole method.  Within an
 * attempt the stage-2 descent runs in chunks of check_every iterations (Adam moments kept
 * in the workspace between chunks, so the iterates equal those of one launch); after each
 * chunk the device orders the particles and, at the first chunk whose end state has a
 * satisfying particle (violation < sat_eps), sets a flag in the workspace that makes the
 * later chunks of the attempt exit at entry.  All chunks of an attempt are enqueued at
 * once and the host reads the outcome once per attempt.  An attempt that reaches K
 * without a satisfying particle is followed by a new one with fresh samples (seed +
 * attempt * 0x9E3779B97F4A7C15), at most max_attempts, and the stage-2 iterations of all
 * attempts together stop at SPASM_TTFS_MAX_ITERS.  The returned particle is the best of
 * the stopping chunk (satisfying first), or of the last attempt.  out->total_ms is device
 * time from the start to the last attempt's result (HIP events); *attempts_out and
 * *iters_out (nullable) receive the attempts and stage-2 iterations run (to the stopping
 * chunk).  Requires K >= 1.  d_work: spasm_solve_ttfs_workspace() bytes, 256-byte
 * aligned. */
#define SPASM_TTFS_MAX_ITERS 30000
size_t spasm_solve_ttfs_workspace(spasm_problem prob, const spasm_solve_config *cfg);
int spasm_solve_ttfs(spasm_problem prob, const spasm_solve_config *cfg, int32_t check_every,
                     int32_t max_attempts, void *d_work, size_t work_bytes, float *d_best_q,
                     float *d_best_pose, spasm_result *out, int32_t *attempts_out, int32_t *iters_out,
                     void *stream);

/* --- serving (continuous batching) --------------------------------------------------------
 * A server owns one device arena of hbm_budget bytes, max_slots solve slots, an
 * admission stream and four class streams.  Requests are queued by spasm_server_submit.
 * Each spasm_server_step:
 *   1. admits queued requests in arrival order while a slot is free and the request's
 *      footprint (spasm_server_footprint) fits in the arena, and runs their stage 1, lift
 *      and seeding on the admission stream, followed there by their first chunk of stage-2
 *      iterations; they join the batched launches from the next step;
 *   2. advances every other running solve by a chunk of stage-2 iterations in ONE launch
 *      per (thread count, sphere chunk) class -- solves of different block counts,
 *      waypoint counts and clutter share a launch, each particle is a workgroup, and the
 *      state stays on the device between steps.  Classes run on separate streams and
 *      overlap.  The slowest class (by measured time per iteration) advances
 *      iters_per_step iterations or 2 ms of work, whichever is more, the others as many
 *      as fit the same time (at most 64 iters_per_step);
 *   3. finishes solves that reached K (final evaluation, best particle written to the
 *      d_best_q [2B][W][7] / d_best_pose [B][4] buffers given at submit time) and queues
 *      their completion records;
 * then synchronises its streams.  A request's result is the same whatever else is in the
 * batch and however its iterations are chunked (every particle runs the same code on its
 * own state).  Not thread-safe: one thread drives a server; the problem and output
 * buffers of a request must stay valid until its completion is polled.
 * spasm_server_submit returns SPASM_EBUSY when the request can never fit
 * (footprint > budget).  max_slots trades latencies: with few slots a large request
 * shares the device with fewer later ones and finishes sooner (tail latency), with many
 * the small requests that arrive behind it start sooner (median latency). */
typedef struct spasm_server_s *spasm_server;

typedef struct {
    uint64_t req_id;
    int32_t status;      /* SPASM_OK, or the error that ended the request */
    int32_t steps;       /* server steps from admission (its prefix step) to completion */
    spasm_result result; /* per-request stage times are not measured (0) */
} spasm_completion;

size_t spasm_server_footprint(spasm_problem prob, const spasm_solve_config *cfg);
int spasm_server_create(size_t hbm_budget, int32_t max_slots, int32_t iters_per_step, spasm_server *out);
int spasm_server_submit(spasm_server srv, spasm_problem prob, const spasm_solve_config *cfg, uint64_t req_id,
                        float *d_best_q, float *d_best_pose);
int spasm_server_step(spasm_server srv, int32_t *n_active, int32_t *n_pending);
int spasm_server_poll(spasm_server srv, spasm_completion *out, int32_t max, int32_t *n_out);
void spasm_server_destroy(spasm_server srv);

const char *spasm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
