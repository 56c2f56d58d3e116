/* FP64 CPU oracle of the SPaSM hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct reference used by the tests, the smoke check and
 * the CPU-baseline leg of the benchmark.  It shares no code or header with the HIP
 * library.  Layouts (all row-major, float64):
 *   stage-1 state  x    [N][B][3]      x, y, yaw per block (z fixed to its slot)
 *   stage-2 state  q    [P][2B][W][7]  segment s = 2b (transit to block b) and
 *                                      s = 2b+1 (transfer of block b)
 *                  pose [P][B][4]      x, y, z, yaw of the placed blocks
 */
#ifndef SPASM_ORACLE_H
#define SPASM_ORACLE_H
#include <stdint.h>

typedef struct {
    int S, O, B, mode;              /* mode 0: tower, 1: fixed goals, 2: packing,
                                       3: point to point (one motion q_home -> p2p_goal,
                                          trajectory [P][1][W][7], endpoints pinned) */
    const double *dh;               /* [7][3] a, d, alpha */
    const double *lo, *hi;          /* [7] */
    double tool_d;
    const double *q_home;           /* [7] */
    const int32_t *sph_link;        /* [S] in 1..7 */
    const double *sph_c;            /* [S][3] link-frame centres */
    const double *sph_r;            /* [S] */
    const double *boxes;            /* [O][6] centre, half extents */
    double h, block_margin;
    const double *block_init;       /* [B][4] */
    const double *goal;             /* [B][4] */
    const double *grasp;            /* [3][4] G: block -> end effector */
    const double *table;            /* [4] */
    const double *w;                /* [9] stable height coll start tie arm block lim smooth */
    const int32_t *pack_cells;      /* [B] cells per piece (mode 2: packing), else NULL */
    const double *pack_off;         /* [B][8][2] cell centres in the piece frame */
    int sample_yaw_steps;           /* stage-1 yaw samples: 0 uniform, n > 0 on n directions */
    const double *p2p_goal;         /* [7] goal configuration (mode 3: point to point) */
} or_problem;

enum { OR_LIN = 0, OR_QUAD = 1 };

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void or_fk(const or_problem *pb, const double *q, double *frames /* [9][12] */);
double or_box_sdf(const double *p, const double *box, double *grad);
double or_obb_sdf(const double *p, const double *pose, double half, double *gp, double *gpose);
double or_square_pen(const double *ca, double tha, const double *cb, double thb, double s, double *g);

void or_place_cost(const or_problem *pb, int dim, int phase, int N, const double *x,
                   double *cost, double *viol, double *grad, double *kink);
void or_traj_cost(const or_problem *pb, int phase, int P, int W, const double *q,
                  const double *pose, double *cost, double *viol, double *gq,
                  double *gpose, double *slot_kink, double *pose_kink);
void or_traj_residuals(const or_problem *pb, int P, int W, const double *q, const double *pose, double *cat);
void or_traj_slot_residuals(const or_problem *pb, int P, int W, const double *q, const double *pose,
                            double *slot_cat);
void or_box_clearance(const or_problem *pb, int W, const double *q, const double *pose, int n,
                      const double *boxes, double *out);
void or_traj_cost_al(const or_problem *pb, int phase, int P, int W, const double *q,
                     const double *pose, const double *lam, double *e_out, double *cost,
                     double *viol, double *gq, double *gpose, double *slot_kink,
                     double *pose_kink);
void or_al_update(const or_problem *pb, int P, const double *e, double rho, double *lam);

void or_schedule(int k, int k_lin, double eta, double alpha, int *phase, double *lr);
void or_gd_step(const or_problem *pb, int N, double *x, const double *g, double lr);
void or_traj_adam_step(const or_problem *pb, int P, int W, double *q, double *pose,
                       double *mq, double *vq, double *mp, double *vp,
                       const double *gq, const double *gpose, double lr, int t,
                       double b1, double b2, double eps);

void or_sample(const or_problem *pb, int N, uint64_t seed, int round, double *x);
void or_argsort(int n, const double *key, int32_t *idx);
void or_order(int n, const double *cost, const double *viol, double eps, int32_t *order,
              int32_t *n_sat);
void or_ik_iterate(const or_problem *pb, int kind, const double *target, double *q,
                   int iters, double lambda);
double or_ik_error(const or_problem *pb, int kind, const double *target, const double *q);
double or_arm_clutter(const or_problem *pb, const double *q, const double *pose, int b, int kind);
void or_ik_lift(const or_problem *pb, int P, const double *pose, uint64_t seed, int iters,
                double lambda, double noise, int restarts, double *q_grasp, double *q_place);
void or_traj_init(const or_problem *pb, int P, int W, const double *q_grasp,
                  const double *q_place, const double *pose, uint64_t seed, double noise,
                  int candidates, double *q);
void or_stage1(const or_problem *pb, int N, int M, uint64_t seed, int round, int k_lin,
               int k_quad, double eta, double alpha, double *x_out, double *cost_out,
               double *viol_out);
void or_stage2(const or_problem *pb, int P, int W, int K, int k_lin, double eta,
               double alpha, double b1, double b2, double eps, double *q, double *pose);
void or_stage2_al(const or_problem *pb, int P, int W, int K, int k_lin, double eta,
                  double alpha, double b1, double b2, double eps, int al_every, double al_rho,
                  double *q, double *pose, double *lam);
#endif
