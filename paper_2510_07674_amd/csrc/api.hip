// C-ABI host side of the SPaSM engine: argument validation, problem packing and
// upload, launch of the device pipeline.  No entry point computes anything on the host.
#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "spasm.h"
#include "spasm_internal.h"

using namespace spasm;
using spasm::fail;

namespace {
thread_local std::string g_err;
std::mutex g_attr_mu;
bool g_attr_done[64];

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

bool valid_W(int W) { return W == 4 || W == 8 || W == 16 || W == 32 || W == 64; }
}  // namespace

namespace spasm {
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Optimiser state per particle: Adam m and v over (2B W 7 joint angles, 4B pose values),
// then, with the augmented Lagrangian, the 15 multipliers of each block.
size_t opt_floats(const KProb &K, int W)
{
    const size_t per = (size_t)2 * K.B * W * NJ + 4 * K.B;
    return 2 * per + (K.al_every > 0 ? (size_t)15 * K.B : 0);
}

void set_opt_layout(const KProb &K, int W, TrajArgs &a)
{
    a.opt_stride = (int)opt_floats(K, W);
    if (K.al_every > 0 && a.opt) {
        a.lam = a.opt + (opt_floats(K, W) - (size_t)15 * K.B);
        a.lam_stride = a.opt_stride;
    }
}

int ensure_attrs()
{
    int dev = 0;
    SPASM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_attr_mu);
    if (dev >= 0 && dev < 64 && !g_attr_done[dev]) {
        SPASM_HIP(set_smem_limits(MAX_SORT * sizeof(unsigned long long), 2 * NJ * MAX_THREADS * sizeof(float)));
        g_attr_done[dev] = true;
    }
    return SPASM_OK;
}

int check_traj_shape(int B, int P, int W)
{
    if (P < 1) return fail(SPASM_EINVAL, "P=%d must be >= 1", P);
    if (!valid_W(W)) return fail(SPASM_EUNSUPPORTED, "W=%d must be 4, 8, 16, 32 or 64", W);
    if (2 * B * W > MAX_THREADS)
        return fail(SPASM_EUNSUPPORTED, "2*B*W=%d exceeds %d waypoint slots per particle", 2 * B * W, MAX_THREADS);
    return SPASM_OK;
}
}  // namespace spasm

extern "C" const char *spasm_last_error(void) { return g_err.c_str(); }

extern "C" int spasm_problem_create(const spasm_chain_desc *chain, int32_t n_sph, const int32_t *sph_link,
                                    const double *sph_c, const double *sph_r, int32_t n_obs, const double *boxes,
                                    const spasm_skeleton_desc *skel, const spasm_params *prm, spasm_problem *out)
{
    if (!out) return fail(SPASM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!chain || !skel || !prm) return fail(SPASM_EINVAL, "chain, skeleton and params are required");
    if (n_sph < 0 || n_obs < 0) return fail(SPASM_EINVAL, "negative sphere or obstacle count");
    if (n_sph > 0 && (!sph_link || !sph_c || !sph_r)) return fail(SPASM_EINVAL, "sphere arrays are NULL");
    if (n_obs > 0 && !boxes) return fail(SPASM_EINVAL, "obstacle array is NULL");
    const int B = skel->n_blocks;
    if (B < 1 || B > MAX_B) return fail(SPASM_EUNSUPPORTED, "n_blocks=%d outside 1..%d", B, MAX_B);
    if (skel->mode != SPASM_MODE_TOWER && skel->mode != SPASM_MODE_FIXED && skel->mode != SPASM_MODE_PACK &&
        skel->mode != SPASM_MODE_P2P)
        return fail(SPASM_EINVAL, "unknown skeleton mode %d", skel->mode);
    if (skel->mode == SPASM_MODE_P2P) {
        if (B != 1) return fail(SPASM_EINVAL, "point-to-point problems take n_blocks = 1 (a placeholder)");
        if (!skel->p2p_goal) return fail(SPASM_EINVAL, "point-to-point problems need p2p_goal");
        if (!finite_all(skel->p2p_goal, 7)) return fail(SPASM_EINVAL, "non-finite p2p_goal");
        for (int j = 0; j < NJ; ++j)
            if (!(chain->q_home[j] >= chain->lo[j] && chain->q_home[j] <= chain->hi[j] &&
                  skel->p2p_goal[j] >= chain->lo[j] && skel->p2p_goal[j] <= chain->hi[j]))
                return fail(SPASM_EINVAL, "joint %d: start or goal outside the limits", j);
    }
    if (skel->sample_yaw_steps < 0 || skel->sample_yaw_steps > 64)
        return fail(SPASM_EINVAL, "sample_yaw_steps=%d outside 0..64", skel->sample_yaw_steps);
    if (skel->mode == SPASM_MODE_PACK) {
        if (!skel->pack_cells || !skel->pack_off) return fail(SPASM_EINVAL, "packing needs pack_cells and pack_off");
        for (int b = 0; b < B; ++b)
            if (skel->pack_cells[b] < 1 || skel->pack_cells[b] > 8)
                return fail(SPASM_EINVAL, "piece %d: %d cells outside 1..8", b, skel->pack_cells[b]);
        if (!finite_all(skel->pack_off, (size_t)B * 16)) return fail(SPASM_EINVAL, "non-finite cell offset");
    }
    if (!skel->block_init && skel->mode != SPASM_MODE_P2P) return fail(SPASM_EINVAL, "block_init is NULL");
    const double zero_init[4] = {0.0, 0.0, 0.0, 0.0};
    const double *block_init = skel->block_init ? skel->block_init : zero_init;  // p2p placeholder
    if (skel->mode == SPASM_MODE_FIXED && !skel->goal) return fail(SPASM_EINVAL, "fixed goals need goal poses");
    if (!finite_all(&chain->dh[0][0], 21) || !finite_all(chain->lo, 7) || !finite_all(chain->hi, 7) ||
        !finite_all(chain->q_home, 7) || !std::isfinite(chain->tool_d))
        return fail(SPASM_EINVAL, "non-finite chain description");
    for (int j = 0; j < NJ; ++j)
        if (!(chain->lo[j] <= chain->hi[j])) return fail(SPASM_EINVAL, "joint %d: lo > hi", j);
    if (n_sph > 0 && (!finite_all(sph_c, (size_t)n_sph * 3) || !finite_all(sph_r, n_sph)))
        return fail(SPASM_EINVAL, "non-finite sphere description");
    for (int i = 0; i < n_sph; ++i) {
        if (sph_link[i] < 1 || sph_link[i] > NJ) return fail(SPASM_EINVAL, "sphere %d: link %d outside 1..7", i, sph_link[i]);
        if (i > 0 && sph_link[i] < sph_link[i - 1]) return fail(SPASM_EINVAL, "sphere links must be non-decreasing");
        if (!(sph_r[i] > 0.0)) return fail(SPASM_EINVAL, "sphere %d: radius must be > 0", i);
    }
    if (n_obs > 0 && !finite_all(boxes, (size_t)n_obs * 6)) return fail(SPASM_EINVAL, "non-finite obstacle");
    for (int o = 0; o < n_obs; ++o)
        for (int c = 3; c < 6; ++c)
            if (boxes[6 * o + c] < 0.0) return fail(SPASM_EINVAL, "obstacle %d: negative half extent", o);
    if (!finite_all(block_init, (size_t)B * 4) ||
        (skel->mode == SPASM_MODE_FIXED && !finite_all(skel->goal, (size_t)B * 4)) ||
        !finite_all(&skel->grasp[0][0], 12) || !finite_all(skel->region, 4) || !std::isfinite(skel->block_edge) ||
        !std::isfinite(skel->block_margin))
        return fail(SPASM_EINVAL, "non-finite skeleton description");
    const double h = skel->block_edge;
    if (!(h > 0.0)) return fail(SPASM_EINVAL, "block_edge must be > 0");
    if (!(skel->block_margin >= 0.0 && skel->block_margin < 0.25 * h)) return fail(SPASM_EINVAL, "block_margin outside [0, h/4)");
    if (!(skel->region[1] - skel->region[0] >= h && skel->region[3] - skel->region[2] >= h))
        return fail(SPASM_EINVAL, "placement region smaller than a block");
    // grasp must be a rigid transform
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double d = 0.0;
            for (int k = 0; k < 3; ++k) d += skel->grasp[k][a] * skel->grasp[k][b];
            if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-6) return fail(SPASM_EINVAL, "grasp rotation is not orthonormal");
        }
    if (!finite_all(prm->w, 9)) return fail(SPASM_EINVAL, "non-finite weights");
    for (int i = 0; i < 9; ++i)
        if (prm->w[i] < 0.0) return fail(SPASM_EINVAL, "negative weight %d", i);
    if (prm->k_lin1 < 0 || prm->k_quad1 < 0 || prm->ik_iters < 0 || prm->retries < 0)
        return fail(SPASM_EINVAL, "negative iteration count");
    if (prm->ik_restarts < 1 || prm->ik_restarts > 8)
        return fail(SPASM_EINVAL, "ik_restarts=%d outside 1..8", prm->ik_restarts);
    if (prm->mid_candidates < 1 || prm->mid_candidates > 8)
        return fail(SPASM_EINVAL, "mid_candidates=%d outside 1..8", prm->mid_candidates);
    if (prm->al_every < 0 || !(prm->al_rho >= 0.0 && std::isfinite(prm->al_rho)))
        return fail(SPASM_EINVAL, "al_every must be >= 0 and al_rho finite and >= 0");
    const double pv[] = {prm->eta1, prm->alpha1, prm->lin_frac2, prm->eta2, prm->alpha2, prm->beta1, prm->beta2,
                         prm->adam_eps, prm->ik_lambda, prm->ik_noise, prm->mid_noise, prm->sat_eps};
    if (!finite_all(pv, sizeof(pv) / sizeof(pv[0]))) return fail(SPASM_EINVAL, "non-finite parameter");
    if (!(prm->beta1 >= 0 && prm->beta1 < 1 && prm->beta2 >= 0 && prm->beta2 < 1 && prm->adam_eps > 0))
        return fail(SPASM_EINVAL, "Adam parameters outside their ranges");
    if (!(prm->lin_frac2 >= 0.0 && prm->lin_frac2 <= 1.0)) return fail(SPASM_EINVAL, "lin_frac2 outside [0, 1]");

    // sphere table, links padded to a multiple of the chunk size
    int count[NJ] = {0};
    for (int i = 0; i < n_sph; ++i) count[sph_link[i] - 1]++;
    int maxper = 0;
    for (int k = 0; k < NJ; ++k) maxper = std::max(maxper, count[k]);
    const int chunk = maxper <= 4 ? 4 : maxper <= 6 ? 6 : maxper == 7 ? 7 : 8;
    std::vector<float> sph;
    int link_start[8];
    link_start[0] = 0;
    {
        int src = 0;
        for (int k = 0; k < NJ; ++k) {
            const int padded = (count[k] + chunk - 1) / chunk * chunk;
            for (int m = 0; m < padded; ++m) {
                if (m < count[k]) {
                    sph.push_back((float)sph_c[3 * src]);
                    sph.push_back((float)sph_c[3 * src + 1]);
                    sph.push_back((float)sph_c[3 * src + 2]);
                    sph.push_back((float)sph_r[src]);
                    ++src;
                } else {  // never overlaps anything
                    sph.push_back(0.f);
                    sph.push_back(0.f);
                    sph.push_back(0.f);
                    sph.push_back(-1e30f);
                }
            }
            link_start[k + 1] = (int)(sph.size() / 4);
        }
    }
    // per box four float4: centre, half extents, lower corner, upper corner (w unused)
    std::vector<float> box((size_t)n_obs * 16, 0.f);
    for (int o = 0; o < n_obs; ++o) {
        for (int c = 0; c < 3; ++c) {
            const double ctr = boxes[6 * o + c], ext = boxes[6 * o + 3 + c];
            box[16 * o + c] = (float)ctr;
            box[16 * o + 4 + c] = (float)ext;
            box[16 * o + 8 + c] = (float)(ctr - ext);
            box[16 * o + 12 + c] = (float)(ctr + ext);
        }
    }
    auto pack_poses = [&](const double *src, std::vector<float> &dst) {
        dst.assign((size_t)B * 8, 0.f);
        for (int b = 0; b < B; ++b) {
            for (int c = 0; c < 4; ++c) dst[8 * b + c] = (float)src[4 * b + c];
            dst[8 * b + 4] = (float)std::cos(src[4 * b + 3]);
            dst[8 * b + 5] = (float)std::sin(src[4 * b + 3]);
        }
    };
    std::vector<float> init, goal, cells((size_t)B * 8 * 4, 0.f);
    pack_poses(block_init, init);
    if (skel->mode == SPASM_MODE_PACK)  // [B][8] (ox, oy, 1 for a cell of the piece, 0)
        for (int b = 0; b < B; ++b)
            for (int k = 0; k < skel->pack_cells[b]; ++k) {
                cells[(b * 8 + k) * 4 + 0] = (float)skel->pack_off[(b * 8 + k) * 2 + 0];
                cells[(b * 8 + k) * 4 + 1] = (float)skel->pack_off[(b * 8 + k) * 2 + 1];
                cells[(b * 8 + k) * 4 + 2] = 1.f;
            }
    if (skel->mode == SPASM_MODE_FIXED)
        pack_poses(skel->goal, goal);
    else
        goal.assign((size_t)B * 8, 0.f);

    const size_t off_sph = 0, n_sphf = sph.size();
    const size_t off_box = align256((off_sph + n_sphf) * 4) / 4, n_boxf = box.size();
    const size_t off_init = align256((off_box + n_boxf) * 4) / 4;
    const size_t off_goal = align256((off_init + init.size()) * 4) / 4;
    const size_t off_cells = align256((off_goal + goal.size()) * 4) / 4;
    const size_t tables = align256((off_cells + cells.size()) * 4);
    const size_t total = tables + align256(sizeof(KProb));  // then the problem struct itself
    std::vector<float> host(tables / 4, 0.f);
    std::copy(sph.begin(), sph.end(), host.begin() + off_sph);
    std::copy(box.begin(), box.end(), host.begin() + off_box);
    std::copy(init.begin(), init.end(), host.begin() + off_init);
    std::copy(goal.begin(), goal.end(), host.begin() + off_goal);
    std::copy(cells.begin(), cells.end(), host.begin() + off_cells);

    auto *pb = new spasm_problem_s();
    if (hipGetDevice(&pb->device) != hipSuccess) {
        delete pb;
        return fail(SPASM_EHIP, "hipGetDevice failed");
    }
    if (hipMalloc(&pb->dmem, total) != hipSuccess) {
        delete pb;
        return fail(SPASM_ENOMEM, "hipMalloc(%zu) failed", total);
    }
    if (hipMemcpy(pb->dmem, host.data(), tables, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(pb->dmem);
        delete pb;
        return fail(SPASM_EHIP, "problem upload failed");
    }
    for (auto &e : pb->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : pb->ev)
                if (f) (void)hipEventDestroy(f);
            (void)hipFree(pb->dmem);
            delete pb;
            return fail(SPASM_EHIP, "hipEventCreate failed");
        }
    float *base = (float *)pb->dmem;
    KProb &K = pb->kp;
    std::memset(&K, 0, sizeof(K));
    K.sph = (const float4 *)(base + off_sph);
    K.box = (const float4 *)(base + off_box);
    K.blk_init = (const float4 *)(base + off_init);
    K.goal = (const float4 *)(base + off_goal);
    K.cells = (const float4 *)(base + off_cells);
    K.self = (const KProb *)((char *)pb->dmem + tables);
    K.yaw_steps = skel->sample_yaw_steps;
    K.lpb_log2 = 3;
    if (skel->mode == SPASM_MODE_PACK) {  // one lane per cell of the largest piece, at least 4
        int mc = 1;
        for (int b = 0; b < B; ++b) mc = std::max(mc, (int)skel->pack_cells[b]);
        K.lpb_log2 = mc <= 4 ? 2 : 3;
    }
    K.al_every = prm->al_every;
    K.al_rho = (float)prm->al_rho;
    if (skel->mode == SPASM_MODE_P2P)
        for (int j = 0; j < NJ; ++j) K.p2p_goal[j] = (float)skel->p2p_goal[j];
    for (int c = 0; c < 4; ++c) K.wall[c] = (float)skel->region[c];
    K.B = B;
    K.S = link_start[7];
    K.O = n_obs;
    K.mode = skel->mode;
    K.chunk = chunk;
    for (int k = 0; k < 8; ++k) K.link_start[k] = link_start[k];
    for (int j = 0; j < NJ; ++j) {
        K.a[j] = (float)chain->dh[j][0];
        K.d[j] = (float)chain->dh[j][1];
        K.ca[j] = (float)std::cos(chain->dh[j][2]);
        K.sa[j] = (float)std::sin(chain->dh[j][2]);
        K.lo[j] = (float)chain->lo[j];
        K.hi[j] = (float)chain->hi[j];
        K.q_home[j] = (float)chain->q_home[j];
    }
    K.tool_d = (float)chain->tool_d;
    K.h = (float)h;
    K.half = (float)(0.5 * h);
    K.r_blk = (float)(0.25 * h - skel->block_margin);
    K.sph_off = (float)(0.25 * h);
    {
        const double xl = skel->region[0] + 0.5 * h, xh = skel->region[1] - 0.5 * h;
        const double yl = skel->region[2] + 0.5 * h, yh = skel->region[3] - 0.5 * h;
        K.samp_x0 = (float)xl;
        K.samp_xs = (float)(xh - xl);
        K.samp_y0 = (float)yl;
        K.samp_ys = (float)(yh - yl);
        K.clamp_xl = (float)xl;
        K.clamp_xh = (float)xh;
        K.clamp_yl = (float)yl;
        K.clamp_yh = (float)yh;
    }
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) K.Gi_R[3 * i + j] = (float)skel->grasp[j][i];
        double t = 0.0;
        for (int k = 0; k < 3; ++k) t -= skel->grasp[k][i] * skel->grasp[k][3];
        K.Gi_t[i] = (float)t;
    }
    for (int i = 0; i < 9; ++i) K.w[i] = (float)prm->w[i];
    K.k_lin1 = prm->k_lin1;
    K.k_quad1 = prm->k_quad1;
    K.eta1 = (float)prm->eta1;
    K.alpha1 = (float)prm->alpha1;
    K.eta2 = (float)prm->eta2;
    K.alpha2 = (float)prm->alpha2;
    K.beta1 = (float)prm->beta1;
    K.beta2 = (float)prm->beta2;
    K.adam_eps = (float)prm->adam_eps;
    K.ik_iters = prm->ik_iters;
    K.ik_restarts = prm->ik_restarts;
    K.mid_candidates = prm->mid_candidates;
    K.ik_lambda = (float)prm->ik_lambda;
    K.ik_noise = (float)prm->ik_noise;
    K.mid_noise = (float)prm->mid_noise;
    K.sat_eps = (float)prm->sat_eps;
    pb->k_total1 = prm->k_lin1 + prm->k_quad1;
    pb->retries = prm->retries;
    pb->lin_frac2 = prm->lin_frac2;
    pb->sat_eps = (float)prm->sat_eps;
    pb->ik_iters = prm->ik_iters;
    if (hipMemcpy((void *)K.self, &K, sizeof(KProb), hipMemcpyHostToDevice) != hipSuccess) {
        spasm_problem_destroy(pb);
        return fail(SPASM_EHIP, "problem upload failed");
    }
    *out = pb;
    return SPASM_OK;
}

extern "C" void spasm_problem_destroy(spasm_problem prob)
{
    if (!prob) return;
    for (auto &e : prob->ev)
        if (e) (void)hipEventDestroy(e);
    if (prob->dmem) (void)hipFree(prob->dmem);
    delete prob;
}

extern "C" int spasm_problem_blocks(spasm_problem prob) { return prob ? prob->kp.B : 0; }

static int check_traj_shape(spasm_problem prob, int P, int W)
{
    if (prob->kp.mode == SPASM_MODE_PACK) return fail(SPASM_EUNSUPPORTED, "packing problems support stage 1 only");
    return spasm::check_traj_shape(prob->kp.B, P, W);
}

extern "C" int spasm_sample(spasm_problem prob, int32_t N, uint64_t seed, int32_t round, float *d_x, void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    if (N < 1 || !d_x) return fail(SPASM_EINVAL, "N must be >= 1 and d_x non-NULL");
    SPASM_HIP(launch_sample(prob->kp, N, seed, round, d_x, nullptr, (hipStream_t)stream));
    return SPASM_OK;
}

extern "C" int spasm_cost_grad(spasm_problem prob, int32_t stage, int32_t phase, int32_t P, int32_t W,
                               const float *d_x, const float *d_pose, float *d_cost, float *d_viol, float *d_gx,
                               float *d_gpose, void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    if (phase != SPASM_PHASE_LIN && phase != SPASM_PHASE_QUAD) return fail(SPASM_EINVAL, "unknown phase %d", phase);
    if (!d_x) return fail(SPASM_EINVAL, "d_x is NULL");
    if (stage == SPASM_STAGE_PLACE) {
        if (P < 1) return fail(SPASM_EINVAL, "P=%d must be >= 1", P);
        SPASM_HIP(launch_place(prob->kp, P, d_x, nullptr, nullptr, 1, 1, phase, d_cost, d_viol, d_gx, nullptr,
                               (hipStream_t)stream));
        return SPASM_OK;
    }
    if (stage != SPASM_STAGE_TRAJ) return fail(SPASM_EINVAL, "unknown stage %d", stage);
    int rc = check_traj_shape(prob, P, W);
    if (rc) return rc;
    if (!d_pose && prob->kp.mode != SPASM_MODE_P2P) return fail(SPASM_EINVAL, "d_pose is NULL");
    TrajArgs a{};
    a.P = P;
    a.W = W;
    a.phase = phase;
    a.q_in = d_x;
    a.pose_in = d_pose;
    a.cost = d_cost;
    a.viol = d_viol;
    a.gq = d_gx;
    a.gpose = d_gpose;
    SPASM_HIP(launch_traj(prob->kp, (d_gx || d_gpose) ? 1 : 0, a, (hipStream_t)stream));
    return SPASM_OK;
}

extern "C" int spasm_cost_adjoint(spasm_problem prob, int32_t phase, int32_t P, int32_t W, const float *d_q,
                                  const float *d_pose, const float *d_gout, float *d_gq, float *d_gpose, void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    if (phase != SPASM_PHASE_LIN && phase != SPASM_PHASE_QUAD) return fail(SPASM_EINVAL, "unknown phase %d", phase);
    int rc = check_traj_shape(prob, P, W);
    if (rc) return rc;
    const bool p2p = prob->kp.mode == SPASM_MODE_P2P;  // no pose variables
    if (!d_q || !d_gout || !d_gq || (!p2p && (!d_pose || !d_gpose))) return fail(SPASM_EINVAL, "NULL buffer");
    TrajArgs a{};
    a.P = P;
    a.W = W;
    a.phase = phase;
    a.q_in = d_q;
    a.pose_in = d_pose;
    a.gout = d_gout;
    a.gq = d_gq;
    a.gpose = d_gpose;
    SPASM_HIP(launch_traj(prob->kp, 1, a, (hipStream_t)stream));
    return SPASM_OK;
}

extern "C" int spasm_cost_grad_al(spasm_problem prob, int32_t phase, int32_t P, int32_t W, const float *d_q,
                                  const float *d_pose, const float *d_lambda, float *d_cost, float *d_viol, float *d_gq,
                                  float *d_gpose, void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    if (phase != SPASM_PHASE_LIN && phase != SPASM_PHASE_QUAD) return fail(SPASM_EINVAL, "unknown phase %d", phase);
    int rc = check_traj_shape(prob, P, W);
    if (rc) return rc;
    if (!d_q || !d_lambda || (!d_pose && prob->kp.mode != SPASM_MODE_P2P)) return fail(SPASM_EINVAL, "NULL buffer");
    TrajArgs a{};
    a.P = P;
    a.W = W;
    a.phase = phase;
    a.q_in = d_q;
    a.pose_in = d_pose;
    a.cost = d_cost;
    a.viol = d_viol;
    a.gq = d_gq;
    a.gpose = d_gpose;
    a.lam = const_cast<float *>(d_lambda);  // read only: no multiplier step outside optimise
    a.lam_stride = 15 * prob->kp.B;
    SPASM_HIP(launch_traj(prob->kp, (d_gq || d_gpose) ? 1 : 0, a, (hipStream_t)stream));
    return SPASM_OK;
}

extern "C" int spasm_optimize(spasm_problem prob, int32_t stage, int32_t P, int32_t W, float *d_x, float *d_pose,
                              float *d_opt, int32_t k_begin, int32_t k_end, int32_t K_total, float *d_cost,
                              float *d_viol, void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    if (!d_x) return fail(SPASM_EINVAL, "d_x is NULL");
    if (k_begin < 1 || k_end < k_begin) return fail(SPASM_EINVAL, "step range [%d, %d) invalid", k_begin, k_end);
    if (stage == SPASM_STAGE_PLACE) {
        if (P < 1) return fail(SPASM_EINVAL, "P=%d must be >= 1", P);
        if (k_end - 1 > prob->k_total1) return fail(SPASM_EINVAL, "stage-1 schedule has %d steps", prob->k_total1);
        SPASM_HIP(launch_place(prob->kp, P, d_x, nullptr, d_x, k_begin, k_end, SPASM_PHASE_QUAD, d_cost, d_viol,
                               nullptr, nullptr, (hipStream_t)stream));
        return SPASM_OK;
    }
    if (stage != SPASM_STAGE_TRAJ) return fail(SPASM_EINVAL, "unknown stage %d", stage);
    int rc = check_traj_shape(prob, P, W);
    if (rc) return rc;
    if (!d_pose && prob->kp.mode != SPASM_MODE_P2P) return fail(SPASM_EINVAL, "d_pose is NULL");
    if (K_total < k_end - 1) return fail(SPASM_EINVAL, "K_total=%d shorter than the step range", K_total);
    rc = ensure_attrs();
    if (rc) return rc;
    if (prob->kp.al_every > 0 && !d_opt)
        return fail(SPASM_EINVAL, "the augmented Lagrangian keeps its multipliers in d_opt: it must not be NULL");
    TrajArgs a{};
    a.P = P;
    a.W = W;
    a.q_in = d_x;
    a.pose_in = d_pose;
    a.q_out = d_x;
    a.pose_out = d_pose;
    a.opt = d_opt;
    set_opt_layout(prob->kp, W, a);
    a.k_begin = k_begin;
    a.k_end = k_end;
    a.k_lin2 = (int)std::lround(prob->lin_frac2 * K_total);
    a.cost = d_cost;
    a.viol = d_viol;
    SPASM_HIP(launch_traj(prob->kp, 2, a, (hipStream_t)stream));
    return SPASM_OK;
}

extern "C" int spasm_select_topm(int32_t N, const float *d_key, int32_t M, int32_t *d_idx, void *stream)
{
    if (N < 1 || N > MAX_SORT) return fail(SPASM_EUNSUPPORTED, "N=%d outside 1..%d", N, MAX_SORT);
    if (M < 1 || M > N) return fail(SPASM_EINVAL, "M=%d outside 1..N", M);
    if (!d_key || !d_idx) return fail(SPASM_EINVAL, "NULL buffer");
    int rc = ensure_attrs();
    if (rc) return rc;
    SPASM_HIP(launch_sort_keys(0, N, d_key, nullptr, 0.f, M, d_idx, nullptr, nullptr, (hipStream_t)stream));
    return SPASM_OK;
}

static int check_topm_shape(int32_t N, int32_t M)
{
    if (N < 1 || N > MAX_TOPM_N) return fail(SPASM_EUNSUPPORTED, "N=%d outside 1..%d", N, MAX_TOPM_N);
    if (M < 1 || M > N) return fail(SPASM_EINVAL, "M=%d outside 1..N", M);
    if (N > MAX_SORT && M > MAX_TOPM_M)
        return fail(SPASM_EUNSUPPORTED, "M=%d above %d for N > %d", M, MAX_TOPM_M, MAX_SORT);
    return SPASM_OK;
}

extern "C" size_t spasm_select_topm_workspace(int32_t N, int32_t M)
{
    if (check_topm_shape(N, M)) return 0;
    return topm_workspace(N, M);
}

extern "C" int spasm_select_topm_large(int32_t N, const float *d_key, int32_t M, int32_t *d_idx, void *d_work,
                                       size_t work_bytes, void *stream)
{
    int rc = check_topm_shape(N, M);
    if (rc) return rc;
    if (!d_key || !d_idx) return fail(SPASM_EINVAL, "NULL buffer");
    const size_t need = topm_workspace(N, M);
    if (work_bytes < need || (need && !d_work))
        return fail(SPASM_EINVAL, "workspace of %zu bytes, %zu needed", work_bytes, need);
    if (need && ((uintptr_t)d_work & 255) != 0) return fail(SPASM_EINVAL, "workspace is not 256-byte aligned");
    rc = ensure_attrs();
    if (rc) return rc;
    SPASM_HIP(launch_topm(N, d_key, M, d_idx, d_work, (hipStream_t)stream));
    return SPASM_OK;
}

namespace {
struct PlaceLayout {
    size_t x1, c1, v1, idx, xs, cs, vs, ord, topm, total;
};
PlaceLayout place_layout(int B, int N, int M)
{
    PlaceLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.x1 = take((size_t)N * B * 3 * sizeof(float));
    L.c1 = take((size_t)N * sizeof(float));
    L.v1 = take((size_t)N * sizeof(float));
    L.idx = take((size_t)M * sizeof(int32_t));
    L.xs = take((size_t)M * B * 3 * sizeof(float));
    L.cs = take((size_t)M * sizeof(float));
    L.vs = take((size_t)M * sizeof(float));
    L.ord = take((size_t)M * sizeof(int32_t));
    L.topm = take(topm_workspace(N, M));
    L.total = o;
    return L;
}
}  // namespace

extern "C" size_t spasm_place_workspace(spasm_problem prob, int32_t N, int32_t M)
{
    if (!prob || check_topm_shape(N, M)) return 0;
    return place_layout(prob->kp.B, N, M).total;
}

extern "C" int spasm_place_round(spasm_problem prob, int32_t N, int32_t M, uint64_t seed, int32_t round, void *d_work,
                                 size_t work_bytes, float *d_x, float *d_cost, float *d_viol, int32_t *d_nsat,
                                 void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    int rc = check_topm_shape(N, M);
    if (rc) return rc;
    if (round < 0) return fail(SPASM_EINVAL, "round=%d must be >= 0", round);
    if (!d_x || !d_nsat) return fail(SPASM_EINVAL, "NULL output buffer");
    const PlaceLayout L = place_layout(prob->kp.B, N, M);
    if (!d_work || work_bytes < L.total) return fail(SPASM_EINVAL, "workspace of %zu bytes, %zu needed", work_bytes, L.total);
    if (((uintptr_t)d_work & 255) != 0) return fail(SPASM_EINVAL, "workspace is not 256-byte aligned");
    rc = ensure_attrs();
    if (rc) return rc;
    const KProb &K = prob->kp;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)d_work;
    auto F = [&](size_t o) { return (float *)(w + o); };
    auto I = [&](size_t o) { return (int32_t *)(w + o); };
    SPASM_HIP(launch_sample(K, N, seed, round, F(L.x1), nullptr, st));
    SPASM_HIP(launch_place(K, N, F(L.x1), nullptr, nullptr, 1, 1, SPASM_PHASE_LIN, F(L.c1), F(L.v1), nullptr, nullptr,
                           st));
    SPASM_HIP(launch_topm(N, F(L.c1), M, I(L.idx), w + L.topm, st));
    SPASM_HIP(launch_place(K, M, F(L.x1), I(L.idx), F(L.xs), 1, prob->k_total1 + 1, SPASM_PHASE_QUAD, F(L.cs), F(L.vs),
                           nullptr, nullptr, st));
    SPASM_HIP(launch_sort_keys(1, M, F(L.cs), F(L.vs), prob->sat_eps, M, I(L.ord), d_nsat, nullptr, st));
    SPASM_HIP(launch_gather_place(K.B, M, F(L.xs), F(L.cs), F(L.vs), I(L.ord), d_x, d_cost, d_viol, st));
    return SPASM_OK;
}

namespace {
struct SampleLayout {
    size_t x1, c1, v1, idx, topm, total;
};
SampleLayout sample_layout(int B, int N, int M)
{
    SampleLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.x1 = take((size_t)N * B * 3 * sizeof(float));
    L.c1 = take((size_t)N * sizeof(float));
    L.v1 = take((size_t)N * sizeof(float));
    L.idx = take((size_t)M * sizeof(int32_t));
    L.topm = take(topm_workspace(N, M));
    L.total = o;
    return L;
}

struct Stage1Layout {
    size_t x1, c1, v1, idx, xs, cs, vs, ord1, nsat1, done, total;
};
Stage1Layout stage1_layout(int B, int N, int M)
{
    Stage1Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.x1 = take((size_t)N * B * 3 * sizeof(float));
    L.c1 = take((size_t)N * sizeof(float));
    L.v1 = take((size_t)N * sizeof(float));
    L.idx = take((size_t)M * sizeof(int32_t));
    L.xs = take((size_t)M * B * 3 * sizeof(float));
    L.cs = take((size_t)M * sizeof(float));
    L.vs = take((size_t)M * sizeof(float));
    L.ord1 = take((size_t)M * sizeof(int32_t));
    L.nsat1 = take(sizeof(int32_t));
    L.done = take(sizeof(int32_t));
    L.total = o;
    return L;
}

int check_stage1_shape(spasm_problem prob, int32_t N, int32_t M)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    if (prob->kp.mode != SPASM_MODE_TOWER && prob->kp.mode != SPASM_MODE_PACK)
        return fail(SPASM_EUNSUPPORTED, "stage 1 places tower or packing blocks (fixed goals and point-to-point "
                                        "problems have none to place)");
    if (M < 1 || N < M || N > MAX_SORT)
        return fail(SPASM_EUNSUPPORTED, "stage 1 needs 1 <= M <= N <= %d (N=%d, M=%d)", MAX_SORT, N, M);
    return SPASM_OK;
}
}  // namespace

extern "C" size_t spasm_sample_placements_workspace(spasm_problem prob, int32_t N, int32_t M)
{
    if (!prob || check_topm_shape(N, M)) return 0;
    return sample_layout(prob->kp.B, N, M).total;
}

extern "C" int spasm_sample_placements(spasm_problem prob, int32_t N, int32_t M, uint64_t seed, int32_t round,
                                       void *d_work, size_t work_bytes, float *d_place, float *d_cost, float *d_viol,
                                       void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    int rc = check_topm_shape(N, M);
    if (rc) return rc;
    if (round < 0) return fail(SPASM_EINVAL, "round=%d must be >= 0", round);
    if (!d_place) return fail(SPASM_EINVAL, "NULL output buffer");
    const SampleLayout L = sample_layout(prob->kp.B, N, M);
    if (!d_work || work_bytes < L.total) return fail(SPASM_EINVAL, "workspace of %zu bytes, %zu needed", work_bytes, L.total);
    if (((uintptr_t)d_work & 255) != 0) return fail(SPASM_EINVAL, "workspace is not 256-byte aligned");
    rc = ensure_attrs();
    if (rc) return rc;
    const KProb &K = prob->kp;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)d_work;
    auto F = [&](size_t o) { return (float *)(w + o); };
    auto I = [&](size_t o) { return (int32_t *)(w + o); };
    SPASM_HIP(launch_sample(K, N, seed, round, F(L.x1), nullptr, st));
    SPASM_HIP(launch_place(K, N, F(L.x1), nullptr, nullptr, 1, 1, SPASM_PHASE_LIN, F(L.c1), F(L.v1), nullptr, nullptr,
                           st));
    SPASM_HIP(launch_topm(N, F(L.c1), M, I(L.idx), w + L.topm, st));
    SPASM_HIP(launch_gather_place(K.B, M, F(L.x1), F(L.c1), F(L.v1), I(L.idx), d_place, d_cost, d_viol, st));
    return SPASM_OK;
}

extern "C" size_t spasm_stage1_workspace(spasm_problem prob, int32_t N, int32_t M)
{
    if (check_stage1_shape(prob, N, M)) return 0;
    return stage1_layout(prob->kp.B, N, M).total;
}

extern "C" int spasm_stage1(spasm_problem prob, int32_t N, int32_t M, uint64_t seed, void *d_work, size_t work_bytes,
                            float *d_pose, float *d_cost, float *d_viol, int32_t *d_info, void *stream)
{
    int rc = check_stage1_shape(prob, N, M);
    if (rc) return rc;
    if (!d_pose || !d_info) return fail(SPASM_EINVAL, "NULL output buffer");
    const Stage1Layout L = stage1_layout(prob->kp.B, N, M);
    if (!d_work || work_bytes < L.total) return fail(SPASM_EINVAL, "workspace of %zu bytes, %zu needed", work_bytes, L.total);
    if (((uintptr_t)d_work & 255) != 0) return fail(SPASM_EINVAL, "workspace is not 256-byte aligned");
    rc = ensure_attrs();
    if (rc) return rc;
    char *w = (char *)d_work;
    auto F = [&](size_t o) { return (float *)(w + o); };
    auto I = [&](size_t o) { return (int32_t *)(w + o); };
    const Stage1Bufs b{F(L.x1), F(L.c1), F(L.v1), I(L.idx), F(L.xs), F(L.cs), F(L.vs), I(L.ord1), I(L.nsat1),
                       I(L.done), d_pose, d_cost, d_viol, d_info};
    return enqueue_stage1(prob, N, M, seed, b, (hipStream_t)stream);
}

extern "C" int spasm_order(int32_t n, const float *d_cost, const float *d_viol, float eps, int32_t *d_order,
                           int32_t *d_nsat, void *stream)
{
    if (n < 1 || n > MAX_SORT) return fail(SPASM_EUNSUPPORTED, "n=%d outside 1..%d", n, MAX_SORT);
    if (!d_cost || !d_viol || !d_order || !d_nsat) return fail(SPASM_EINVAL, "NULL buffer");
    if (!std::isfinite(eps)) return fail(SPASM_EINVAL, "eps must be finite");
    int rc = ensure_attrs();
    if (rc) return rc;
    SPASM_HIP(launch_sort_keys(1, n, d_cost, d_viol, eps, n, d_order, d_nsat, nullptr, (hipStream_t)stream));
    return SPASM_OK;
}

extern "C" int spasm_ik_iterate(spasm_problem prob, int32_t kind, int32_t n, const float *d_target, float *d_q,
                                int32_t iters, void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    if (prob->kp.mode == SPASM_MODE_PACK) return fail(SPASM_EUNSUPPORTED, "packing problems support stage 1 only");
    if (prob->kp.mode == SPASM_MODE_P2P) return fail(SPASM_EUNSUPPORTED, "point-to-point problems have no blocks to grasp");
    if (kind != 0 && kind != 1) return fail(SPASM_EINVAL, "kind must be 0 (grasp) or 1 (place)");
    if (n < 1 || iters < 0 || !d_target || !d_q) return fail(SPASM_EINVAL, "bad size or NULL buffer");
    SPASM_HIP(launch_ik_iterate(prob->kp, kind, n, d_target, d_q, iters, (hipStream_t)stream));
    return SPASM_OK;
}

extern "C" int spasm_ik_lift(spasm_problem prob, int32_t P, const float *d_pose, uint64_t seed, int32_t iters,
                             float *d_qgrasp, float *d_qplace, void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    if (prob->kp.mode == SPASM_MODE_PACK) return fail(SPASM_EUNSUPPORTED, "packing problems support stage 1 only");
    if (prob->kp.mode == SPASM_MODE_P2P) return fail(SPASM_EUNSUPPORTED, "point-to-point problems have no blocks to grasp");
    if (P < 1 || iters < 0 || !d_pose || !d_qgrasp || !d_qplace) return fail(SPASM_EINVAL, "bad size or NULL buffer");
    SPASM_HIP(launch_ik_lift(prob->kp, P, d_pose, seed, iters, d_qgrasp, d_qplace, (hipStream_t)stream));
    return SPASM_OK;
}

extern "C" int spasm_traj_init(spasm_problem prob, int32_t P, int32_t W, const float *d_qgrasp, const float *d_qplace,
                               const float *d_pose, uint64_t seed, float *d_q, void *stream)
{
    if (!prob) return fail(SPASM_EINVAL, "problem is NULL");
    int rc = check_traj_shape(prob, P, W);
    if (rc) return rc;
    if (!d_q || (prob->kp.mode != SPASM_MODE_P2P && (!d_qgrasp || !d_qplace || !d_pose)))
        return fail(SPASM_EINVAL, "NULL buffer");
    SPASM_HIP(launch_traj_init(prob->kp, P, W, d_qgrasp, d_qplace, d_pose, seed, d_q, (hipStream_t)stream));
    return SPASM_OK;
}

// ---------------------------------------------------------------------------------------
// whole method
// ---------------------------------------------------------------------------------------
namespace {
__global__ void k_zero_words(uint32_t *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}
}  // namespace

namespace spasm {
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t *)p, n);
    return hipGetLastError();
}

SolveLayout solve_layout(const KProb &K, const spasm_solve_config &c)
{
    SolveLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t B = K.B, M = c.M, N1 = c.N1, W = c.W;
    if (N1 > 0) {
        L.x1 = take(N1 * B * 3 * 4);
        L.c1 = take(N1 * 4);
        L.v1 = take(N1 * 4);
        L.idx = take(M * 4);
        L.xs = take(M * B * 3 * 4);
        L.cs = take(M * 4);
        L.vs = take(M * 4);
        L.ord1 = take(M * 4);
        L.nsat1 = take(4);
        L.done = take(4);
    }
    L.pose = take(M * B * 4 * 4);
    if (K.al_every > 0) L.lam = take(M * B * 15 * 4);
    L.qg = take(M * B * NJ * 4);
    L.qp = take(M * B * NJ * 4);
    L.q = take(M * 2 * B * W * NJ * 4);
    L.c2 = take(M * 4);
    L.v2 = take(M * 4);
    L.ord2 = take(M * 4);
    L.nsat2 = take(4);
    L.info = take(8 * 4);
    L.finfo = take(4 * 4);
    L.total = off;
    return L;
}

int check_cfg(spasm_problem prob, const spasm_solve_config *cfg)
{
    if (!prob || !cfg) return fail(SPASM_EINVAL, "problem and config are required");
    if (prob->kp.mode == SPASM_MODE_PACK)
        return fail(SPASM_EUNSUPPORTED, "packing problems support stage 1 only (place_round)");
    if (cfg->M < 1 || cfg->M > MAX_SORT) return fail(SPASM_EUNSUPPORTED, "M=%d outside 1..%d", cfg->M, MAX_SORT);
    if (prob->kp.mode == SPASM_MODE_TOWER) {
        if (cfg->N1 < cfg->M || cfg->N1 > MAX_SORT)
            return fail(SPASM_EUNSUPPORTED, "towers need M <= N1 <= %d (N1=%d)", MAX_SORT, cfg->N1);
    } else if (cfg->N1 != 0) {
        return fail(SPASM_EINVAL, "fixed-goal and point-to-point problems take N1 = 0");
    }
    if (cfg->K < 0) return fail(SPASM_EINVAL, "K must be >= 0");
    return check_traj_shape(prob->kp.B, cfg->M, cfg->W);
}

// Alg. 1 lines 1-23 on the device: rounds of sample -> linear score -> top-M -> descent ->
// satisfying-first order, each round skipped (kernels exit at once) after a round has
// committed; a round commits when it has a satisfying particle or is the last one.
int enqueue_stage1(spasm_problem prob, int N1, int M, uint64_t seed, const Stage1Bufs &b, hipStream_t st)
{
    const KProb &K = prob->kp;
    SPASM_HIP(launch_zero(b.done, 4, st));
    SPASM_HIP(launch_zero(b.info, 8, st));
    const int R = prob->retries;
    for (int r = 0; r <= R; ++r) {
        const int *skip = b.done;
        SPASM_HIP(launch_sample(K, N1, seed, r, b.x1, skip, st));
        SPASM_HIP(launch_place(K, N1, b.x1, nullptr, nullptr, 1, 1, SPASM_PHASE_LIN, b.c1, b.v1, nullptr, skip, st));
        SPASM_HIP(launch_sort_keys(0, N1, b.c1, nullptr, 0.f, M, b.idx, nullptr, skip, st));
        SPASM_HIP(launch_place(K, M, b.x1, b.idx, b.xs, 1, prob->k_total1 + 1, SPASM_PHASE_QUAD, b.cs, b.vs, nullptr,
                               skip, st));
        SPASM_HIP(launch_sort_keys(1, M, b.cs, b.vs, prob->sat_eps, M, b.ord1, b.nsat1, skip, st));
        SPASM_HIP(launch_commit_stage1(K, M, r, r == R, b.xs, b.cs, b.vs, b.ord1, b.nsat1, b.pose, b.cost_out,
                                       b.viol_out, b.done, b.info, st));
    }
    return SPASM_OK;
}

int enqueue_prefix(spasm_problem prob, const spasm_solve_config &cfg, char *w, const SolveLayout &L, hipStream_t st,
                   hipEvent_t after_stage1)
{
    const KProb &K = prob->kp;
    auto F = [&](size_t o) { return (float *)(w + o); };
    auto I = [&](size_t o) { return (int32_t *)(w + o); };
    const int M = cfg.M, W = cfg.W;
    if (cfg.N1 > 0) {
        SPASM_HIP(launch_zero(I(L.info), 32, st));
        const Stage1Bufs b{F(L.x1), F(L.c1), F(L.v1), I(L.idx), F(L.xs), F(L.cs), F(L.vs), I(L.ord1), I(L.nsat1),
                           I(L.done), F(L.pose), nullptr, nullptr, I(L.info)};
        const int rc = enqueue_stage1(prob, cfg.N1, M, cfg.seed, b, st);
        if (rc) return rc;
    } else {
        SPASM_HIP(launch_fixed_poses(K, M, F(L.pose), I(L.info), st));
    }
    if (after_stage1) SPASM_HIP(hipEventRecord(after_stage1, st));
    if (K.mode != SPASM_MODE_P2P)  // a point-to-point motion has its ends already
        SPASM_HIP(launch_ik_lift(K, M, F(L.pose), cfg.seed, prob->ik_iters, F(L.qg), F(L.qp), st));
    SPASM_HIP(launch_traj_init(K, M, W, F(L.qg), F(L.qp), F(L.pose), cfg.seed, F(L.q), st));
    return SPASM_OK;
}

int enqueue_finish(spasm_problem prob, const spasm_solve_config &cfg, char *w, const SolveLayout &L, float *best_q,
                   float *best_pose, hipStream_t st)
{
    const KProb &K = prob->kp;
    auto F = [&](size_t o) { return (float *)(w + o); };
    auto I = [&](size_t o) { return (int32_t *)(w + o); };
    SPASM_HIP(launch_sort_keys(1, cfg.M, F(L.c2), F(L.v2), prob->sat_eps, cfg.M, I(L.ord2), I(L.nsat2), nullptr, st));
    SPASM_HIP(launch_finalize(K, cfg.M, cfg.W, F(L.q), F(L.pose), F(L.c2), F(L.v2), I(L.ord2), I(L.nsat2), best_q,
                              best_pose, I(L.info), F(L.finfo), st));
    return SPASM_OK;
}
}  // namespace spasm

extern "C" size_t spasm_solve_workspace(spasm_problem prob, const spasm_solve_config *cfg)
{
    if (check_cfg(prob, cfg)) return 0;
    return solve_layout(prob->kp, *cfg).total;
}

extern "C" size_t spasm_solve_footprint(spasm_problem prob, const spasm_solve_config *cfg)
{
    if (check_cfg(prob, cfg)) return 0;
    const KProb &K = prob->kp;
    const size_t ns = K.mode == SPASM_MODE_P2P ? 1 : 2 * (size_t)K.B;
    return align256(solve_layout(K, *cfg).total) + align256(ns * cfg->W * NJ * sizeof(float)) +
           align256((size_t)K.B * 4 * sizeof(float));
}

namespace spasm {
size_t stage2_opt_bytes(const KProb &K, const spasm_solve_config &cfg)
{
    return (size_t)cfg.M * opt_floats(K, cfg.W) * sizeof(float);
}
}  // namespace spasm

// When a solve's particles need more waves than the chip holds at once (4 waves of 128
// VGPRs per SIMD), workgroups start as others finish and a costly particle started late
// sets the end of the launch: rank the seeded particles by one cost-only evaluation (into
// cost) so that the fused kernel takes them costliest first (longest processing time
// first).  Every particle computes the same thing on whichever workgroup runs it.  Sets
// a.perm to perm, or leaves it null when every particle is resident anyway.
static int order_costliest_first(spasm_problem prob, const spasm_solve_config &cfg, const float *q, const float *pose,
                                 float *cost, int32_t *perm, TrajArgs &a, hipStream_t st)
{
    const KProb &K = prob->kp;
    int cus = 0;
    SPASM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, prob->device));
    const long waves = (long)cfg.M * (traj_threads(K.B, cfg.W) / 64);
    if (waves <= 16L * cus || cfg.M > MAX_SORT) return SPASM_OK;
    TrajArgs e{};
    e.P = cfg.M;
    e.W = cfg.W;
    e.phase = 0;
    e.q_in = q;
    e.pose_in = pose;
    e.cost = cost;
    SPASM_HIP(launch_traj(K, 0, e, st));
    SPASM_HIP(launch_sort_keys(0, cfg.M, cost, nullptr, 0.f, cfg.M, perm, nullptr, nullptr, st));
    a.perm = perm;
    return SPASM_OK;
}

extern "C" size_t spasm_solve_ttfs_workspace(spasm_problem prob, const spasm_solve_config *cfg)
{
    if (check_cfg(prob, cfg)) return 0;
    return align256(solve_layout(prob->kp, *cfg).total) + align256(stage2_opt_bytes(prob->kp, *cfg)) +
           align256((size_t)cfg->M * sizeof(int32_t)) + 256;
}

extern "C" int spasm_solve_ttfs(spasm_problem prob, const spasm_solve_config *cfg, int32_t check_every,
                                int32_t max_attempts, void *d_work, size_t work_bytes, float *d_best_q,
                                float *d_best_pose, spasm_result *out, int32_t *attempts_out, int32_t *iters_out,
                                void *stream)
{
    int rc = check_cfg(prob, cfg);
    if (rc) return rc;
    if (check_every < 1) return fail(SPASM_EINVAL, "check_every=%d must be >= 1", check_every);
    if (max_attempts < 1) return fail(SPASM_EINVAL, "max_attempts=%d must be >= 1", max_attempts);
    if (cfg->K < 1) return fail(SPASM_EINVAL, "time to first solution needs K >= 1");
    if (!d_work || !d_best_q || !d_best_pose || !out) return fail(SPASM_EINVAL, "NULL buffer");
    if (((uintptr_t)d_work & 255) != 0) return fail(SPASM_EINVAL, "workspace must be 256-byte aligned");
    const KProb &K = prob->kp;
    const SolveLayout L = solve_layout(K, *cfg);
    const size_t opt_off = align256(L.total), obytes = stage2_opt_bytes(K, *cfg);
    const size_t perm_off = opt_off + align256(obytes);
    const size_t flag_off = perm_off + align256((size_t)cfg->M * sizeof(int32_t)), need = flag_off + 256;
    if (work_bytes < need) return fail(SPASM_EINVAL, "workspace %zu bytes < %zu needed", work_bytes, need);
    rc = ensure_attrs();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)d_work;
    auto F = [&](size_t o) { return (float *)(w + o); };
    auto I = [&](size_t o) { return (int32_t *)(w + o); };
    int32_t *done = I(flag_off), *stop_iter = done + 1;

    SPASM_HIP(hipEventRecord(prob->ev[0], st));
    int att = 0, iters = 0;
    int32_t info[8] = {0}, flags[2] = {0, 0};
    float finfo[4] = {0.f};
    bool solved = false;
    for (att = 0; att < max_attempts && !solved && iters < SPASM_TTFS_MAX_ITERS; ++att) {
        spasm_solve_config ca = *cfg;
        ca.seed = cfg->seed + (uint64_t)att * 0x9E3779B97F4A7C15ull;  // fresh samples per attempt
        rc = enqueue_prefix(prob, ca, w, L, st);
        if (rc) return rc;
        SPASM_HIP(launch_zero(w + opt_off, obytes, st));
        SPASM_HIP(launch_zero(done, 8, st));
        TrajArgs a{};
        a.P = ca.M;
        a.W = ca.W;
        a.q_in = F(L.q);
        a.pose_in = F(L.pose);
        a.q_out = F(L.q);
        a.pose_out = F(L.pose);
        a.opt = F(opt_off);
        set_opt_layout(K, ca.W, a);
        a.k_lin2 = (int)std::lround(prob->lin_frac2 * ca.K);
        a.cost = F(L.c2);
        a.viol = F(L.v2);
        a.skip = done;
        rc = order_costliest_first(prob, ca, F(L.q), F(L.pose), F(L.c2), I(perm_off), a, st);
        if (rc) return rc;
        // every chunk is enqueued at once; after the first chunk whose end state has a
        // satisfying particle the device sets `done` and the later chunks exit at entry
        const int k_last = std::min(ca.K, SPASM_TTFS_MAX_ITERS - iters);
        for (int k0 = 1; k0 <= k_last; k0 += check_every) {
            a.k_begin = k0;
            a.k_end = std::min(k_last, k0 + check_every - 1) + 1;
            SPASM_HIP(launch_traj(K, 2, a, st));
            SPASM_HIP(launch_sort_keys(1, ca.M, F(L.c2), F(L.v2), prob->sat_eps, ca.M, I(L.ord2), I(L.nsat2), done, st));
            SPASM_HIP(launch_check_stop(I(L.nsat2), done, stop_iter, a.k_end - 1, st));
        }
        SPASM_HIP(launch_finalize(K, ca.M, ca.W, F(L.q), F(L.pose), F(L.c2), F(L.v2), I(L.ord2), I(L.nsat2),
                                  d_best_q, d_best_pose, I(L.info), F(L.finfo), st));
        SPASM_HIP(hipMemcpyAsync(info, I(L.info), sizeof(info), hipMemcpyDeviceToHost, st));
        SPASM_HIP(hipMemcpyAsync(finfo, F(L.finfo), sizeof(finfo), hipMemcpyDeviceToHost, st));
        SPASM_HIP(hipMemcpyAsync(flags, done, sizeof(flags), hipMemcpyDeviceToHost, st));
        SPASM_HIP(hipEventRecord(prob->ev[1], st));
        SPASM_HIP(hipStreamSynchronize(st));  // one host check per attempt
        solved = flags[0] != 0;
        iters += solved ? flags[1] : k_last;
    }
    float t = 0.f;
    SPASM_HIP(hipEventElapsedTime(&t, prob->ev[0], prob->ev[1]));
    std::memset(out, 0, sizeof(*out));
    out->stage1_sat = info[0];
    out->rounds = info[1];
    out->n_sat = info[2];
    out->best = info[3];
    out->success = info[2] > 0;
    out->viol = finfo[0];
    out->cost = finfo[1];
    out->length = finfo[2];
    out->total_ms = t;
    if (attempts_out) *attempts_out = att;
    if (iters_out) *iters_out = iters;
    return SPASM_OK;
}

extern "C" int spasm_solve(spasm_problem prob, const spasm_solve_config *cfg, void *d_work, size_t work_bytes,
                           float *d_best_q, float *d_best_pose, spasm_result *out, void *stream)
{
    int rc = check_cfg(prob, cfg);
    if (rc) return rc;
    if (!d_work || !d_best_q || !d_best_pose || !out) return fail(SPASM_EINVAL, "NULL buffer");
    if (((uintptr_t)d_work & 255) != 0) return fail(SPASM_EINVAL, "workspace must be 256-byte aligned");
    const KProb &K = prob->kp;
    const SolveLayout L = solve_layout(K, *cfg);
    if (work_bytes < L.total) return fail(SPASM_EINVAL, "workspace %zu bytes < %zu needed", work_bytes, L.total);
    rc = ensure_attrs();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)d_work;
    auto F = [&](size_t o) { return (float *)(w + o); };
    auto I = [&](size_t o) { return (int32_t *)(w + o); };

    hipEvent_t *ev = prob->ev;

    SPASM_HIP(hipEventRecord(ev[0], st));
    rc = enqueue_prefix(prob, *cfg, w, L, st, ev[1]);
    if (rc) return rc;
    TrajArgs a{};
    a.P = cfg->M;
    a.W = cfg->W;
    a.q_in = F(L.q);
    a.pose_in = F(L.pose);
    a.q_out = F(L.q);
    a.pose_out = F(L.pose);
    a.k_begin = 1;
    a.k_end = cfg->K + 1;
    a.k_lin2 = (int)std::lround(prob->lin_frac2 * cfg->K);
    a.cost = F(L.c2);
    a.viol = F(L.v2);
    if (K.al_every > 0) {  // multipliers start at zero
        SPASM_HIP(launch_zero(I(L.lam), (size_t)cfg->M * K.B * 15 * sizeof(float), st));
        a.lam = F(L.lam);
        a.lam_stride = 15 * K.B;
    }
    rc = order_costliest_first(prob, *cfg, F(L.q), F(L.pose), F(L.c2), I(L.ord2), a, st);
    if (rc) return rc;
    SPASM_HIP(hipEventRecord(ev[3], st));
    SPASM_HIP(launch_traj(K, 2, a, st));
    SPASM_HIP(hipEventRecord(ev[4], st));
    rc = enqueue_finish(prob, *cfg, w, L, d_best_q, d_best_pose, st);
    if (rc) return rc;
    SPASM_HIP(hipEventRecord(ev[2], st));
    int32_t info[8];
    float finfo[4];
    SPASM_HIP(hipMemcpyAsync(info, I(L.info), sizeof(info), hipMemcpyDeviceToHost, st));
    SPASM_HIP(hipMemcpyAsync(finfo, F(L.finfo), sizeof(finfo), hipMemcpyDeviceToHost, st));
    SPASM_HIP(hipStreamSynchronize(st));
    float t01 = 0.f, t12 = 0.f, t02 = 0.f, t34 = 0.f;
    SPASM_HIP(hipEventElapsedTime(&t34, ev[3], ev[4]));
    SPASM_HIP(hipEventElapsedTime(&t01, ev[0], ev[1]));
    SPASM_HIP(hipEventElapsedTime(&t12, ev[1], ev[2]));
    SPASM_HIP(hipEventElapsedTime(&t02, ev[0], ev[2]));
    out->stage1_sat = info[0];
    out->rounds = info[1];
    out->n_sat = info[2];
    out->best = info[3];
    out->success = info[2] > 0;
    out->viol = finfo[0];
    out->cost = finfo[1];
    out->length = finfo[2];
    out->stage1_ms = t01;
    out->stage2_ms = t12;
    out->total_ms = t02;
    out->opt_ms = t34;
    return SPASM_OK;
}
