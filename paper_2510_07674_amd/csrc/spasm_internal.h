// Internal declarations shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "spasm.h"

namespace spasm {

constexpr int NJ = 7;           // joints of the serial chain
constexpr int MAX_B = 16;       // blocks per problem
constexpr int MAX_THREADS = 1024;
constexpr int MAX_SORT = 16384; // single-workgroup sort capacity (LDS bound)
constexpr int MAX_TOPM_N = 1 << 20;  // radix-select top-M: keys
constexpr int MAX_TOPM_M = MAX_SORT / 2;  // radix-select top-M: selected keys

// Problem constants passed BY VALUE to every kernel: they land in the kernel-argument
// segment and are read into scalar registers, so every lane of a wave shares one copy.
// Arrays live in device memory and are indexed with wave-uniform indices (scalar loads).
struct KProb {
    const float4 *sph;       // [S] link-frame centre xyz, radius; sorted by link
    const float4 *box;       // [O][2] (cx, cy, cz, 0), (hx, hy, hz, 0)
    const float4 *blk_init;  // [B][2] (x, y, z, yaw), (cos yaw, sin yaw, 0, 0)
    const float4 *goal;      // [B][2] same layout (fixed goals)
    const float4 *cells;     // [B][8] packing cells (ox, oy, 1, 0); (0, 0, 0, 0) past a piece's last cell
    const KProb *self;       // this struct's copy in device memory (for non-inlined device functions)
    int B, S, O, mode;
    int yaw_steps;           // stage-1 yaw samples on yaw_steps directions (0: uniform)
    int lpb_log2;            // stage-1 lanes per block: 8 block spheres (3); packing: cells rounded up to 2^k >= 4
    float wall[4];           // packing walls: region x_lo, x_hi, y_lo, y_hi
    float p2p_goal[NJ];      // point-to-point goal configuration (the start is q_home)
    int al_every;            // augmented Lagrangian: multiplier step every al_every iterations (0: off)
    float al_rho;            // multiplier step al_rho * 2w * residual
    int chunk;               // spheres tested per box fetch (4, 6, 7 or 8); links padded to it
    int link_start[8];       // spheres of link k are [link_start[k-1], link_start[k])
    float a[NJ], d[NJ], ca[NJ], sa[NJ], lo[NJ], hi[NJ], q_home[NJ];
    float tool_d, h, half, r_blk, sph_off;
    float samp_x0, samp_xs, samp_y0, samp_ys;      // sample: x = x0 + xs * u
    float clamp_xl, clamp_xh, clamp_yl, clamp_yh;  // stage-1 clamp box
    float Gi_R[9], Gi_t[3];  // G^-1 (row-major rotation, translation)
    float w[9];              // stable height coll start tie arm block lim smooth
    int k_lin1, k_quad1;
    float eta1, alpha1;
    float eta2, alpha2, beta1, beta2, adam_eps;
    int ik_iters, ik_restarts, mid_candidates;
    float ik_lambda, ik_noise, mid_noise, sat_eps;
};

enum { W_STABLE = 0, W_HEIGHT, W_COLL, W_START, W_TIE, W_ARM, W_BLOCK, W_LIM, W_SMOOTH };

// ---- launchers (kernels.hip).  All enqueue on `st` and return the launch status. ----
// `skip` (nullable, device int): when *skip != 0 the kernel returns immediately; used for
// the device-side stage-1 retry rounds.
hipError_t launch_sample(const KProb &P, int N, uint64_t seed, int round, float *x,
                         const int *skip, hipStream_t st);

// Stage-1 placement kernel: optional gather (x_in rows idx[p]), steps k_begin..k_end-1 of
// gradient descent, then an evaluation at `eval_phase` writing cost/viol/grad.
hipError_t launch_place(const KProb &P, int n, const float *x_in, const int32_t *idx, float *x_out,
                        int k_begin, int k_end, int eval_phase, float *cost, float *viol, float *gx,
                        const int *skip, hipStream_t st);

struct TrajArgs {
    int P, W, phase;
    const float *q_in;
    const float *pose_in;
    float *q_out;       // optimise: final trajectory (may alias q_in)
    float *pose_out;
    float *opt;         // optimise: Adam moments in/out, nullable (zeros, not written)
    int k_begin, k_end, k_lin2;
    const float *gout;  // adjoint scale per particle (nullable)
    float *cost, *viol; // nullable
    float *gq, *gpose;  // nullable
    // augmented-Lagrangian multipliers [particle][B][15] at lam + p * lam_stride (nullable:
    // plain penalties); optimise updates them every P.al_every iterations
    float *lam;
    int lam_stride;
    int opt_stride;     // floats per particle in opt (0: the two moment blocks only)
    // nullable: particle order of the workgroups, particle perm[P - 1 - w] on workgroup w
    // (the solve passes its particles sorted by ascending initial cost, so the launch
    // starts with the costliest)
    const int32_t *perm;
    // nullable device flag: when *skip != 0 the launch returns at once (time to first
    // solution: chunks after the one that found a solution)
    const int32_t *skip;
};
// mode 0: cost only, 1: cost + gradient (scaled by gout if given), 2: optimise
hipError_t launch_traj(const KProb &P, int mode, const TrajArgs &a, hipStream_t st);

// One active solve in a serving launch: its problem, its stage-2 state and the steps of
// this launch; workgroups [first, first + a.P) of the launch are its particles.
struct ServeSolve {
    KProb P;
    TrajArgs a;
    int first;
    int pad[3];
};
// nwg = total particles of the class; d_solves sorted by `first`, device memory
hipError_t launch_serve(int chunk, int threads, int nwg, const ServeSolve *d_solves, int nsolve, hipStream_t st);
int traj_threads(int B, int W);
// optimiser state floats per particle (Adam moments, then multipliers when al_every > 0)
size_t opt_floats(const KProb &K, int W);
void set_opt_layout(const KProb &K, int W, TrajArgs &a);
// raise the dynamic-LDS ceilings of the sort and optimise kernels
hipError_t set_smem_limits(size_t sort_bytes, size_t traj_bytes);

hipError_t launch_sort_keys(int kind, int n, const float *cost, const float *viol, float eps,
                            int M, int32_t *out_idx, int32_t *out_count, const int *skip,
                            hipStream_t st);
size_t topm_workspace(int n, int M);
// Adam moments of a chunked stage-2 run: [M][(2B W 7 + 4B) * 2] floats
size_t stage2_opt_bytes(const KProb &K, const spasm_solve_config &cfg);
hipError_t launch_topm(int n, const float *cost, int M, int32_t *out_idx, void *ws, hipStream_t st);
hipError_t launch_gather_place(int B, int M, const float *xs, const float *cs, const float *vs, const int32_t *ord,
                               float *x_out, float *c_out, float *v_out, hipStream_t st);

hipError_t launch_ik_iterate(const KProb &P, int kind, int n, const float *target, float *q,
                             int iters, hipStream_t st);
hipError_t launch_ik_lift(const KProb &P, int nP, const float *pose, uint64_t seed, int iters,
                          float *qg, float *qp, hipStream_t st);
hipError_t launch_traj_init(const KProb &P, int nP, int W, const float *qg, const float *qp, const float *pose,
                            uint64_t seed, float *q, hipStream_t st);

// solve glue
// Commits round `round` of stage 1 when no earlier round did and it has a satisfying
// particle or is the last: pose[m] = placement xs[order[m]] at its slot height, cost_out /
// viol_out (nullable) the matching cs / vs, *done = 1, info[0] = nsat, info[1] = rounds.
hipError_t launch_commit_stage1(const KProb &P, int M, int round, int last_round, const float *xs,
                                const float *cs, const float *vs, const int32_t *order, const int32_t *nsat,
                                float *pose, float *cost_out, float *viol_out, int *done, int32_t *info,
                                hipStream_t st);
hipError_t launch_fixed_poses(const KProb &P, int M, float *pose, int32_t *info, hipStream_t st);
hipError_t launch_finalize(const KProb &P, int M, int W, const float *q, const float *pose,
                           const float *cost, const float *viol, const int32_t *order,
                           const int32_t *nsat, float *best_q, float *best_pose, int32_t *info,
                           float *finfo, hipStream_t st);

// ---- shared host helpers (api.hip) ----
int fail(int code, const char *fmt, ...);  // records the thread-local message, returns code
size_t align256(size_t x);
int ensure_attrs();
int check_traj_shape(int B, int P, int W);

// Workspace layout of one solve (offsets in bytes from the workspace base).
struct SolveLayout {
    size_t x1, c1, v1, idx, xs, cs, vs, ord1, nsat1, done, pose, lam, qg, qp, q, c2, v2, ord2, nsat2, info, finfo, total;
};
SolveLayout solve_layout(const KProb &K, const spasm_solve_config &c);
int check_cfg(spasm_problem prob, const spasm_solve_config *cfg);
// Stage-1 buffers: samples, their scores, the kept indices, the descended placements and
// their order (working), then the committed outputs (pose [M][B][4]; cost_out, viol_out
// nullable) and the summary info[0..1]; done is the device flag that skips later rounds.
struct Stage1Bufs {
    float *x1, *c1, *v1;
    int32_t *idx;
    float *xs, *cs, *vs;
    int32_t *ord1, *nsat1;
    int32_t *done;
    float *pose, *cost_out, *viol_out;
    int32_t *info;
};
int enqueue_stage1(spasm_problem prob, int N1, int M, uint64_t seed, const Stage1Bufs &b, hipStream_t st);
// Stage 1 (or fixed goals), lift and seeding into the workspace, on `st`.
// after_stage1 (nullable) is recorded between stage 1 and the lift.
int enqueue_prefix(spasm_problem prob, const spasm_solve_config &cfg, char *w, const SolveLayout &L, hipStream_t st,
                   hipEvent_t after_stage1 = nullptr);
// Final ordering, best particle copied to best_q / best_pose, summary in info/finfo.
int enqueue_finish(spasm_problem prob, const spasm_solve_config &cfg, char *w, const SolveLayout &L,
                   float *best_q, float *best_pose, hipStream_t st);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
// Time to first solution: after a chunk's ordering, when *done == 0 and *nsat > 0, sets
// *done = 1 and *stop_iter = iters (the stage-2 iterations run so far in the attempt).
hipError_t launch_check_stop(const int32_t *nsat, int32_t *done, int32_t *stop_iter, int iters, hipStream_t st);

}  // namespace spasm

struct spasm_problem_s {
    spasm::KProb kp;
    void *dmem = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // the solves' timing events
    int device = 0;
    int k_total1 = 0;
    int retries = 0;
    double lin_frac2 = 0.0;
    float sat_eps = 1e-3f;
    int ik_iters = 0;
};

#define SPASM_HIP(expr)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return spasm::fail(SPASM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
