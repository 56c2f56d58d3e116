// gfx950 kernels of the SPaSM hot path (Chen, Iyer, Kingston, arXiv 2510.07674).
//
// Work mapping (wave64, no matrix cores: nothing here is a dense contraction):
//   stage 1   one lane per (particle, block, block-sphere); 8 lanes per block reduce the
//             block's pose gradient with lane shuffles, the particle's poses sit in LDS.
//   stage 2   one workgroup per particle, one lane per waypoint slot (2B segments x W).
//             Obstacle boxes and robot spheres are read with wave-uniform indices (scalar
//             loads into SGPRs); block poses come from an LDS table.  The gradient is
//             formed in reverse mode from per-link wrenches: a force f at point c on link
//             l adds z_{j-1} . ((c - o_{j-1}) x f) to dC/dq_j for every j <= l.
//   optimise  the whole schedule runs inside one launch with the state on chip
//             (trajectory in VGPRs, Adam moments and poses in LDS).
#include <algorithm>

#include "spasm_internal.h"

namespace spasm {

// ------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float sgnf(float x) { return x >= 0.f ? 1.f : -1.f; }

// The problem tables are never written while a kernel runs.  Reading them through the
// constant address space lets the compiler use scalar loads for wave-uniform indices
// even after workgroup barriers (which otherwise count as possible writers).
typedef __attribute__((address_space(4))) const float cfloat;
__device__ __forceinline__ float4 ldc(const float4 *p, int i)
{
    cfloat *q = (cfloat *)(p + i);
    return make_float4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ float phi(int phase, float d) { return phase ? d * d : d; }
__device__ __forceinline__ float dphi(int phase, float d) { return phase ? 2.f * d : 1.f; }

// Target centre height of block b (tower slot, fixed goal, or on the table for packing
// pieces).  Computed, not read from an array in the kernel argument: a per-lane index
// into the by-value argument would force the whole argument into per-lane scratch memory.
__device__ __forceinline__ float zstar(const KProb &P, int b)
{
    if (P.mode == SPASM_MODE_PACK) return 0.5f * P.h;
    return P.mode == 0 ? ((float)b + 0.5f) * P.h : ldc(P.goal, 2 * b).z;
}

// Motion segments per particle: transit and transfer per block, or the single motion of
// a point-to-point problem.
__device__ __forceinline__ int n_segments(const KProb &P) { return P.mode == SPASM_MODE_P2P ? 1 : 2 * P.B; }

// Cross-lane reductions without LDS: DPP within each 16-lane row (quad_perm xor 1 and
// xor 2, row_mirror, row_half_mirror) and the gfx950 row swaps across rows (xor 32, then
// xor 16).  Every step combines a lane with its partner in the same operand order on
// both sides, so all 64 lanes end with bit-identical results, also for sums.
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
struct OpSum {
    __device__ __forceinline__ float operator()(float a, float b) const { return a + b; }
};
struct OpMin {
    __device__ __forceinline__ float operator()(float a, float b) const { return fminf(a, b); }
};
struct OpMax {
    __device__ __forceinline__ float operator()(float a, float b) const { return fmaxf(a, b); }
};
// within groups of 8 lanes (xor 1, xor 2, then quad q with quad q ^ 1 through the half-row
// mirror)
template <class Op>
__device__ __forceinline__ float group8_reduce(float v, Op op)
{
    v = op(v, dpp<0xB1>(v));   // quad_perm [1,0,3,2]
    v = op(v, dpp<0x4E>(v));   // quad_perm [2,3,0,1]
    return op(v, dpp<0x141>(v));  // row_half_mirror
}
template <class Op>
__device__ __forceinline__ float wave_reduce(float v, Op op)
{
    v = group8_reduce(v, op);
    v = op(v, dpp<0x140>(v));  // row_mirror: half-row h with 1 - h
    const int b = __float_as_int(v);
    const auto s32 = __builtin_amdgcn_permlane32_swap(b, b, false, false);
    v = op(__int_as_float(s32[0]), __int_as_float(s32[1]));
    const int c = __float_as_int(v);
    const auto s16 = __builtin_amdgcn_permlane16_swap(c, c, false, false);
    return op(__int_as_float(s16[0]), __int_as_float(s16[1]));
}
// whole-wave shifts by one lane (lane i reads i + 1, resp. i - 1); the end lane keeps its value
__device__ __forceinline__ float lane_next(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
// within each 32-lane half of the wave
template <class Op>
__device__ __forceinline__ float half_reduce(float v, Op op)
{
    v = group8_reduce(v, op);
    v = op(v, dpp<0x140>(v));  // row_mirror
    const int c = __float_as_int(v);
    const auto s16 = __builtin_amdgcn_permlane16_swap(c, c, false, false);
    return op(__int_as_float(s16[0]), __int_as_float(s16[1]));
}
__device__ __forceinline__ float wave_sum(float v) { return wave_reduce(v, OpSum()); }
__device__ __forceinline__ float wave_min(float v) { return wave_reduce(v, OpMin()); }
__device__ __forceinline__ float wave_max(float v) { return wave_reduce(v, OpMax()); }
__device__ __forceinline__ float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Alg. 1 schedule: eta_k = eta (1 - k / k_lin) on the linear cost for k <= k_lin, then the
// fixed rate alpha on the quadratic cost.
__device__ __forceinline__ void schedule(int k, int k_lin, float eta, float alpha, int &phase, float &lr)
{
    if (k <= k_lin) {
        phase = 0;
        lr = eta * (1.f - (float)k / (float)k_lin);
    } else {
        phase = 1;
        lr = alpha;
    }
}

// Philox4x64-10 (Salmon et al., SC'11); 24-bit uniforms.
__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}
__device__ __forceinline__ void uniforms4(uint64_t seed, uint64_t a, uint64_t b, uint64_t c, uint64_t stream,
                                          float u[4])
{
    uint64_t x[4] = {a, b, c, stream};
    philox4x64(x, seed, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = (float)(x[i] >> 40) * (1.0f / 16777216.0f);
}

// Rigid frame: rotation columns x, y, z and origin p.
struct Frame {
    float x0, x1, x2, y0, y1, y2, z0, z1, z2, p0, p1, p2;
};
__device__ __forceinline__ void frame_identity(Frame &F)
{
    F.x0 = 1.f; F.x1 = 0.f; F.x2 = 0.f;
    F.y0 = 0.f; F.y1 = 1.f; F.y2 = 0.f;
    F.z0 = 0.f; F.z1 = 0.f; F.z2 = 1.f;
    F.p0 = 0.f; F.p1 = 0.f; F.p2 = 0.f;
}
// T <- T Rz(q) Tz(d) Tx(a) Rx(alpha)  (classic DH)
__device__ __forceinline__ void dh_step(Frame &F, float a, float d, float ca, float sa, float q)
{
    float s, c;
    sincosf(q, &s, &c);
    const float nx0 = c * F.x0 + s * F.y0, nx1 = c * F.x1 + s * F.y1, nx2 = c * F.x2 + s * F.y2;
    const float u0 = c * F.y0 - s * F.x0, u1 = c * F.y1 - s * F.x1, u2 = c * F.y2 - s * F.x2;
    const float ny0 = ca * u0 + sa * F.z0, ny1 = ca * u1 + sa * F.z1, ny2 = ca * u2 + sa * F.z2;
    const float nz0 = ca * F.z0 - sa * u0, nz1 = ca * F.z1 - sa * u1, nz2 = ca * F.z2 - sa * u2;
    F.p0 += a * nx0 + d * F.z0;
    F.p1 += a * nx1 + d * F.z1;
    F.p2 += a * nx2 + d * F.z2;
    F.x0 = nx0; F.x1 = nx1; F.x2 = nx2;
    F.y0 = ny0; F.y1 = ny1; F.y2 = ny2;
    F.z0 = nz0; F.z1 = nz1; F.z2 = nz2;
}

// Box signed distance from the offsets d = p - centre and u = |d| - half extents:
// outside |max(u,0)| with gradient sgn(d) max(u,0)/|max(u,0)|; inside the largest u with
// the axis of the first largest component.
__device__ __forceinline__ float box_sdf(float dx, float dy, float dz, float ux, float uy, float uz,
                                         float &gx, float &gy, float &gz)
{
    const float qx = fmaxf(ux, 0.f), qy = fmaxf(uy, 0.f), qz = fmaxf(uz, 0.f);
    const float qq = qx * qx + qy * qy + qz * qz;
    if (qq > 0.f) {
        // hardware reciprocal square root (about 1 ulp) instead of the correctly rounded
        // sqrt and divide sequences; qq > 0 here
        const float inv = __builtin_amdgcn_rsqf(qq), n = qq * inv;
        gx = sgnf(dx) * (qx * inv);
        gy = sgnf(dy) * (qy * inv);
        gz = sgnf(dz) * (qz * inv);
        return n;
    }
    if (ux >= uy && ux >= uz) {
        gx = sgnf(dx); gy = 0.f; gz = 0.f;
        return ux;
    }
    if (uy >= uz) {
        gx = 0.f; gy = sgnf(dy); gz = 0.f;
        return uy;
    }
    gx = 0.f; gy = 0.f; gz = sgnf(dz);
    return uz;
}

// ------------------------------------------------------------------------------------
// Sphere sets against obstacles (axis-aligned boxes) and blocks (yawed cubes from the
// LDS pose table), CH spheres per lane at a time.
//
// Obstacles, broad phase: the chunk's spheres over the wave's active lanes are bounded by
// one axis-aligned box (exact min/max, 1e-4 m margin against rounding, held in SGPRs);
// each lane tests one obstacle against it and a ballot keeps the obstacles that overlap.
// A skipped obstacle cannot touch any sphere of the wave.
// Narrow phase per kept obstacle (parameters in SGPRs): a slab test per sphere, which is
// necessary for penetration (sdf >= max(|d| - e)), gives one ballot mask per sphere; the
// exact distance and gradient run only for the spheres that some lane's slab test hits.
// ------------------------------------------------------------------------------------
template <bool GRAD>
__device__ __forceinline__ void contact(int phase, float wgt, float cx, float cy, float cz, float sdf, float r,
                                        float gx, float gy, float gz, float &cost, float &viol, float (&wf)[3],
                                        float (&wt)[3])
{
    const float delta = r - sdf;
    cost += wgt * phi(phase, delta);
    viol = fmaxf(viol, delta);
    if (GRAD) {
        const float sc = -wgt * dphi(phase, delta);
        const float fx = sc * gx, fy = sc * gy, fz = sc * gz;
        wf[0] += fx;
        wf[1] += fy;
        wf[2] += fz;
        wt[0] += cy * fz - cz * fy;
        wt[1] += cz * fx - cx * fz;
        wt[2] += cx * fy - cy * fx;
    }
}

// Axis-aligned bounds of one lane's sphere chunk with a 1e-4 m margin against rounding;
// empty for inactive lanes.
struct LaneBox {
    float lo0, lo1, lo2, hi0, hi1, hi2;
};
template <int CH>
__device__ __forceinline__ LaneBox lane_box(const float (&cx)[CH], const float (&cy)[CH], const float (&cz)[CH],
                                            const float (&r)[CH], bool act)
{
    LaneBox b{INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    if (act) {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            b.lo0 = fminf(b.lo0, cx[i] - r[i]);
            b.lo1 = fminf(b.lo1, cy[i] - r[i]);
            b.lo2 = fminf(b.lo2, cz[i] - r[i]);
            b.hi0 = fmaxf(b.hi0, cx[i] + r[i]);
            b.hi1 = fmaxf(b.hi1, cy[i] + r[i]);
            b.hi2 = fmaxf(b.hi2, cz[i] + r[i]);
        }
        b.lo0 -= 1e-4f;
        b.lo1 -= 1e-4f;
        b.lo2 -= 1e-4f;
        b.hi0 += 1e-4f;
        b.hi1 += 1e-4f;
        b.hi2 += 1e-4f;
    }
    return b;
}

// Narrow-phase passes (sphere chunks tested exactly against one box) of each wave in the
// current stage-2 iteration.  A particle's waves meet at barriers every iteration, so the
// wave with the most contacts sets its particle's pace, and the launch ends with the
// slowest particle; that wave takes a higher issue priority on its SIMD for the next
// iteration (see traj_particle).
// Narrow-phase passes per priority level (levels 0..3): 24 where a CU holds several
// particles (their waves compete for the SIMDs), 8 (PRIO_STEP_HB) for the particles of
// 9-12 waves that have a CU to themselves (measured on 4- and 10-block towers).
__shared__ int s_wave_work[16];
constexpr int PRIO_STEP = 24, PRIO_STEP_HB = 8;

template <bool GRAD, int CH, bool HB = false>
__device__ __forceinline__ void collide_boxes(const KProb &P, int phase, float wgt, const float (&cx)[CH],
                                              const float (&cy)[CH], const float (&cz)[CH], const float (&r)[CH],
                                              const LaneBox &lb, bool act, float &cost, float &viol, float (&wf)[3],
                                              float (&wt)[3])
{
    const int lane = threadIdx.x & 63;
    // broad-phase bounds: the wave's union (lo, hi) or, with HB, one box per half wave
    // (lo, hi for lanes 0-31 and mo, mh for lanes 32-63; a half wave is one segment of 32
    // waypoints, so two segments far apart do not make everything between them a candidate)
    float lo0, lo1, lo2, hi0, hi1, hi2, mo0 = 0.f, mo1 = 0.f, mo2 = 0.f, mh0 = 0.f, mh1 = 0.f, mh2 = 0.f;
    if constexpr (HB) {
        auto rl = [](float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); };
        const float a0 = half_reduce(lb.lo0, OpMin()), a1 = half_reduce(lb.lo1, OpMin());
        const float a2 = half_reduce(lb.lo2, OpMin());
        const float b0 = half_reduce(lb.hi0, OpMax()), b1 = half_reduce(lb.hi1, OpMax());
        const float b2 = half_reduce(lb.hi2, OpMax());
        lo0 = rl(a0, 0);
        lo1 = rl(a1, 0);
        lo2 = rl(a2, 0);
        hi0 = rl(b0, 0);
        hi1 = rl(b1, 0);
        hi2 = rl(b2, 0);
        mo0 = rl(a0, 32);
        mo1 = rl(a1, 32);
        mo2 = rl(a2, 32);
        mh0 = rl(b0, 32);
        mh1 = rl(b1, 32);
        mh2 = rl(b2, 32);
    } else {
        lo0 = uniform(wave_min(lb.lo0));
        lo1 = uniform(wave_min(lb.lo1));
        lo2 = uniform(wave_min(lb.lo2));
        hi0 = uniform(wave_max(lb.hi0));
        hi1 = uniform(wave_max(lb.hi1));
        hi2 = uniform(wave_max(lb.hi2));
    }
    int nar = 0;  // wave-uniform
    for (int base = 0; base < P.O; base += 64) {
        const int ol = base + lane;
        bool ov = false;
        if (ol < P.O) {
            const float4 bl = ldc(P.box, 4 * ol + 2), bh = ldc(P.box, 4 * ol + 3);
            ov = (bl.x <= hi0) & (bh.x >= lo0) & (bl.y <= hi1) & (bh.y >= lo1) & (bl.z <= hi2) & (bh.z >= lo2);
            if constexpr (HB)
                ov |= (bl.x <= mh0) & (bh.x >= mo0) & (bl.y <= mh1) & (bh.y >= mo1) & (bl.z <= mh2) & (bh.z >= mo2);
        }
        unsigned long long m = __ballot(ov);
        while (m) {
            const int o = base + __builtin_ctzll(m);
            m &= m - 1;
            // lane pretest: the lane's own bounds against the obstacle (bitwise &, so the
            // compares stay branch-free and combine as lane masks)
            const float4 bl = ldc(P.box, 4 * o + 2), bh = ldc(P.box, 4 * o + 3);
            const unsigned long long lpm =
                __ballot((lb.lo0 <= bh.x) & (lb.hi0 >= bl.x) & (lb.lo1 <= bh.y) & (lb.hi1 >= bl.y) &
                         (lb.lo2 <= bh.z) & (lb.hi2 >= bl.z));
            if (!lpm) continue;
            const float4 bc = ldc(P.box, 4 * o), be = ldc(P.box, 4 * o + 1);
            unsigned long long hm[CH], any = 0;
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const float ux = fabsf(cx[i] - bc.x) - be.x;
                const float uy = fabsf(cy[i] - bc.y) - be.y;
                const float uz = fabsf(cz[i] - bc.z) - be.z;
                hm[i] = __ballot(fmaxf(fmaxf(ux, uy), uz) < r[i]) & lpm;
                any |= hm[i];
            }
            if (!any) continue;
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                if (!hm[i]) continue;
                ++nar;
                const float dx = cx[i] - bc.x, dy = cy[i] - bc.y, dz = cz[i] - bc.z;
                const float ux = fabsf(dx) - be.x, uy = fabsf(dy) - be.y, uz = fabsf(dz) - be.z;
                float gx, gy, gz;
                const float sdf = box_sdf(dx, dy, dz, ux, uy, uz, gx, gy, gz);
                if (act && r[i] - sdf > 0.f)
                    contact<GRAD>(phase, wgt, cx[i], cy[i], cz[i], sdf, r[i], gx, gy, gz, cost, viol, wf, wt);
            }
        }
    }
    if (nar && lane == 0) s_wave_work[threadIdx.x >> 6] += nar;
}

// Blocks as they stand while the lane's segment runs: b' < b at the placement variable
// (table 0, gradient flows to the pose), b' > b at the initial pose (table 1), block b
// itself at its initial pose only for arm spheres during the transit before the grasp.
template <bool GRAD, int CH>
__device__ __forceinline__ void collide_blocks(const KProb &P, int phase, float wgt, const float (&cx)[CH],
                                               const float (&cy)[CH], const float (&cz)[CH], const float (&r)[CH],
                                               const LaneBox &lb, bool act, int b, bool own_visible,
                                               const float *s_pose, float *s_pacc, float &cost, float &viol,
                                               float (&wf)[3], float (&wt)[3])
{
    const int B = P.B;
    const float half = P.half;
    for (int bb = 0; bb < B; ++bb) {
        const bool movable = bb < b;
        const float *pp = s_pose + ((movable ? 0 : MAX_B) + bb) * 8;
        const float tx = pp[0], ty = pp[1], tz = pp[2], cs = pp[4], sn = pp[5], ext = pp[6];
        // lane pretest against the block's axis-aligned bounds (xy half extent of the
        // yawed square in pp[6])
        const bool vis = act & (bb != b || own_visible) & (tx - ext <= lb.hi0) & (tx + ext >= lb.lo0) &
                         (ty - ext <= lb.hi1) & (ty + ext >= lb.lo1) & (tz - half <= lb.hi2) & (tz + half >= lb.lo2);
        const unsigned long long vm = __ballot(vis);
        if (!vm) continue;
        unsigned long long hm[CH], any = 0;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const float dx = cx[i] - tx, dy = cy[i] - ty, dz = cz[i] - tz;
            const float lx = cs * dx + sn * dy, ly = cs * dy - sn * dx;
            const float ux = fabsf(lx) - half, uy = fabsf(ly) - half, uz = fabsf(dz) - half;
            hm[i] = __ballot(fmaxf(fmaxf(ux, uy), uz) < r[i]) & vm;
            any |= hm[i];
        }
        if (!any) continue;
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (!hm[i]) continue;
            const float dx = cx[i] - tx, dy = cy[i] - ty, dz = cz[i] - tz;
            const float lx = cs * dx + sn * dy, ly = cs * dy - sn * dx;
            const float ux = fabsf(lx) - half, uy = fabsf(ly) - half, uz = fabsf(dz) - half;
            float gx, gy, gz;
            const float sdf = box_sdf(lx, ly, dz, ux, uy, uz, gx, gy, gz);
            if (vis && r[i] - sdf > 0.f) {
                const float wx = cs * gx - sn * gy, wy = sn * gx + cs * gy;  // world gradient
                contact<GRAD>(phase, wgt, cx[i], cy[i], cz[i], sdf, r[i], wx, wy, gz, cost, viol, wf, wt);
                if (GRAD && movable) {
                    const float sc = -wgt * dphi(phase, r[i] - sdf);
                    g0 -= sc * wx;
                    g1 -= sc * wy;
                    g2 -= sc * gz;
                    g3 += sc * (gx * ly - gy * lx);
                }
            }
        }
        if (GRAD) {
            if (__any(g0 != 0.f || g1 != 0.f || g2 != 0.f || g3 != 0.f)) {
                g0 = wave_sum(g0);
                g1 = wave_sum(g1);
                g2 = wave_sum(g2);
                g3 = wave_sum(g3);
                if ((threadIdx.x & 63) == 0) {
                    float *acc = s_pacc + bb * 4;
                    acc[0] += g0;
                    acc[1] += g1;
                    acc[2] += g2;
                    acc[3] += g3;
                }
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// Placement cost lane (Appendix B, tower): sphere k of block i.  The lane owns the cost
// of its sphere against obstacles, blocks placed above it (j > i, pose variables) and
// blocks not moved yet (j > i, initial poses), and for k == 0 the height term and the
// stability term of block i.  It returns the gradient with respect to block i's pose
// (x, y, z, yaw) including the contributions of terms owned by other lanes (the pairs
// (sphere of j < i, box i) and the stability terms of blocks below i), so that a sum
// over the block's 8 lanes gives d cost / d pose_i without any scatter.
// st: LDS pose table of the particle [B][8] = x, y, z, yaw, cos, sin.
// ------------------------------------------------------------------------------------
template <bool GRAD>
__device__ __forceinline__ void place_lane(const KProb &P, int phase, int i, int k, const float *st, float &cost, float &viol,
                           float (&g)[4])
{
    const int B = P.B;
    const float w_coll = P.w[W_COLL], so = P.sph_off, rb = P.r_blk, half = P.half;
    const float sbx = (k & 1) ? so : -so, sby = (k & 2) ? so : -so, sbz = (k & 4) ? so : -so;
    const float xi = st[i * 8 + 0], yi = st[i * 8 + 1], zi = st[i * 8 + 2], ci = st[i * 8 + 4],
                si = st[i * 8 + 5];
    const float cx = xi + ci * sbx - si * sby, cy = yi + si * sbx + ci * sby, cz = zi + sbz;
    const float dyx = -si * sbx - ci * sby, dyy = ci * sbx - si * sby;  // d c / d yaw

    for (int o = 0; o < P.O; ++o) {
        const float4 bc = ldc(P.box, 4 * o), be = ldc(P.box, 4 * o + 1);
        const float dx = cx - bc.x, dy = cy - bc.y, dz = cz - bc.z;
        const float ux = fabsf(dx) - be.x, uy = fabsf(dy) - be.y, uz = fabsf(dz) - be.z;
        if (fmaxf(fmaxf(ux, uy), uz) < rb) {
            float gx, gy, gz;
            const float delta = rb - box_sdf(dx, dy, dz, ux, uy, uz, gx, gy, gz);
            if (delta > 0.f) {
                cost += w_coll * phi(phase, delta);
                viol = fmaxf(viol, delta);
                if (GRAD) {
                    const float sc = -w_coll * dphi(phase, delta);
                    g[0] += sc * gx;
                    g[1] += sc * gy;
                    g[2] += sc * gz;
                    g[3] += sc * (gx * dyx + gy * dyy);
                }
            }
        }
    }
    for (int j = 0; j < B; ++j) {
        // this sphere against block j > i, placed (table) and at its initial pose
#pragma unroll
        for (int tgt = 0; tgt < 2; ++tgt) {
            float tx, ty, tz, cs, sn;
            if (tgt == 0) {
                tx = st[j * 8 + 0]; ty = st[j * 8 + 1]; tz = st[j * 8 + 2]; cs = st[j * 8 + 4]; sn = st[j * 8 + 5];
            } else {
                const float4 a0 = ldc(P.blk_init, 2 * j), a1 = ldc(P.blk_init, 2 * j + 1);
                tx = a0.x; ty = a0.y; tz = a0.z; cs = a1.x; sn = a1.y;
            }
            const float dx = cx - tx, dy = cy - ty, dz = cz - tz;
            const float lx = cs * dx + sn * dy, ly = cs * dy - sn * dx;
            const float ux = fabsf(lx) - half, uy = fabsf(ly) - half, uz = fabsf(dz) - half;
            if (j > i && fmaxf(fmaxf(ux, uy), uz) < rb) {
                float gx, gy, gz;
                const float delta = rb - box_sdf(lx, ly, dz, ux, uy, uz, gx, gy, gz);
                if (delta > 0.f) {
                    cost += w_coll * phi(phase, delta);
                    viol = fmaxf(viol, delta);
                    if (GRAD) {
                        const float sc = -w_coll * dphi(phase, delta);
                        const float wx = cs * gx - sn * gy, wy = sn * gx + cs * gy;
                        g[0] += sc * wx;
                        g[1] += sc * wy;
                        g[2] += sc * gz;
                        g[3] += sc * (wx * dyx + wy * dyy);
                    }
                }
            }
        }
        // sphere k of block j < i against block i: gradient through block i's pose
        if (GRAD && j < i) {
            const float xj = st[j * 8 + 0], yj = st[j * 8 + 1], zj = st[j * 8 + 2], cj = st[j * 8 + 4],
                        sj = st[j * 8 + 5];
            const float px = xj + cj * sbx - sj * sby, py = yj + sj * sbx + cj * sby, pz = zj + sbz;
            const float dx = px - xi, dy = py - yi, dz = pz - zi;
            const float lx = ci * dx + si * dy, ly = ci * dy - si * dx;
            const float ux = fabsf(lx) - half, uy = fabsf(ly) - half, uz = fabsf(dz) - half;
            if (fmaxf(fmaxf(ux, uy), uz) < rb) {
                float gx, gy, gz;
                const float delta = rb - box_sdf(lx, ly, dz, ux, uy, uz, gx, gy, gz);
                if (delta > 0.f) {
                    const float sc = -w_coll * dphi(phase, delta);
                    const float wx = ci * gx - si * gy, wy = si * gx + ci * gy;
                    g[0] -= sc * wx;
                    g[1] -= sc * wy;
                    g[2] -= sc * gz;
                    g[3] += sc * (gx * ly - gy * lx);
                }
            }
        }
    }
    if (k == 0) {
        const float w_h = P.w[W_HEIGHT], w_s = P.w[W_STABLE];
        const float e = zi - zstar(P, i);
        cost += w_h * e * e;
        viol = fmaxf(viol, fabsf(e));
        if (GRAD) g[2] += 2.f * w_h * e;
        if (P.mode == 0) {
            // C_stable terms m <= i: term m compares the mean xy of blocks above m with
            // block m's h x h footprint
            for (int m = 0; m + 1 < B; ++m) {
                if (m > i) break;
                float mx = 0.f, my = 0.f;
                for (int j = m + 1; j < B; ++j) {
                    mx += st[j * 8 + 0];
                    my += st[j * 8 + 1];
                }
                const float n = (float)(B - 1 - m);
                mx /= n;
                my /= n;
                const float cm = st[m * 8 + 4], sm = st[m * 8 + 5];
                const float ex = mx - st[m * 8 + 0], ey = my - st[m * 8 + 1];
                const float v0 = cm * ex + sm * ey, v1 = cm * ey - sm * ex;
                const float a0 = fmaxf(fabsf(v0) - half, 0.f), a1 = fmaxf(fabsf(v1) - half, 0.f);
                const float D = sqrtf(a0 * a0 + a1 * a1);
                if (m == i) {
                    cost += w_s * phi(phase, D);
                    viol = fmaxf(viol, D);
                }
                if (GRAD && D > 0.f) {
                    const float gw = w_s * dphi(phase, D);
                    const float dv0 = sgnf(v0) * a0 / D, dv1 = sgnf(v1) * a1 / D;
                    const float dm0 = cm * dv0 - sm * dv1, dm1 = sm * dv0 + cm * dv1;
                    if (m == i) {
                        g[0] -= gw * dm0;
                        g[1] -= gw * dm1;
                        g[3] += gw * (dv0 * v1 - dv1 * v0);
                    } else {
                        g[0] += gw * dm0 / n;
                        g[1] += gw * dm1 / n;
                    }
                }
            }
        }
    }
}

// Packing placement cost of a whole particle, each cell pair evaluated once.  Lane (i, k)
// holds cell k of piece i.  Its cell's world centre and yaw derivative go to LDS; piece i
// then takes the pairs with pieces j = i + t (mod B), t = 1..floor(B/2) (for t = B/2 only
// when i < j), so every unordered pair of pieces is met once and the pieces share the
// work evenly.  A pair's cost and both pieces' gradients come from that one evaluation:
// the gradient with respect to piece j is what j's own lane would compute (its normals
// first in the choice of the separating axis, d -> -d); it is summed over i's lanes and
// left in LDS per (i, t), and after a barrier each piece adds the contributions left
// for it in fixed order of t.  Called by every lane of the workgroup (barriers inside).
template <bool GRAD>
__device__ __forceinline__ void pack_particle(const KProb &P, int phase, int i, int k, int L, const float *st,
                                              float4 *s_cell, float *s_gj, float &cost, float &viol,
                                              float (&g)[4])
{
    const int B = P.B, T = B >> 1;
    const float w = P.w[W_COLL], s = P.half;
    if (k == 0) {  // height: zero while z stays on the table
        const float w_h = P.w[W_HEIGHT];
        const float e = st[i * 8 + 2] - zstar(P, i);
        cost += w_h * e * e;
        viol = fmaxf(viol, fabsf(e));
        if (GRAD) g[2] += 2.f * w_h * e;
    }
    const float4 ck = ldc(P.cells, 8 * i + k);
    const bool valid = ck.z != 0.f;
    const float xi = st[i * 8 + 0], yi = st[i * 8 + 1], ci = st[i * 8 + 4], si = st[i * 8 + 5];
    const float ax = xi + ci * ck.x - si * ck.y, ay = yi + si * ck.x + ci * ck.y;
    const float dax = -si * ck.x - ci * ck.y, day = ci * ck.x - si * ck.y;  // d(ax, ay) / d yaw_i
    // cells past a piece's last one sit far away, so they never overlap anything
    s_cell[i * L + k] = valid ? make_float4(ax, ay, dax, day) : make_float4(1e30f, 1e30f, 0.f, 0.f);
    __syncthreads();
    if (valid) {
        // walls: the cell reaches e = s (|cos| + |sin|) from its centre along x and along y
        const float e = s * (fabsf(ci) + fabsf(si));
        const float de = s * (sgnf(si) * ci - sgnf(ci) * si);  // d e / d yaw_i
        const float wd[4] = {P.wall[0] - (ax - e), (ax + e) - P.wall[1], P.wall[2] - (ay - e), (ay + e) - P.wall[3]};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (wd[q] > 0.f) {
                cost += w * phi(phase, wd[q]);
                viol = fmaxf(viol, wd[q]);
                if (GRAD) {
                    const float sc = w * dphi(phase, wd[q]);
                    const float sgn = (q & 1) ? 1.f : -1.f;  // inward side: -1 for x_lo / y_lo
                    if (q < 2) {
                        g[0] += sc * sgn;
                        g[3] += sc * (sgn * dax + de);
                    } else {
                        g[1] += sc * sgn;
                        g[3] += sc * (sgn * day + de);
                    }
                }
            }
        }
    }
    for (int t = 1; t <= T; ++t) {
        int j = i + t;
        if (j >= B) j -= B;
        const bool take = valid && (2 * t < B || i < j);
        const float cj = st[j * 8 + 4], sj = st[j * 8 + 5];
        const float cD = cj * ci + sj * si, sD = sj * ci - cj * si;  // cos, sin of yaw_j - yaw_i
        const float R = s * (1.f + fabsf(cD) + fabsf(sD));
        const float dR = s * (sgnf(cD) * sD - sgnf(sD) * cD);      // d R / d yaw_i
        const float dRj = s * (sgnf(cD) * -sD - sgnf(-sD) * cD);   // d R / d yaw_j
        float h0 = 0.f, h1 = 0.f, h3 = 0.f;  // gradient with respect to piece j
        for (int m = 0; m < L; ++m) {
            const float4 cb = s_cell[j * L + m];
            const float dx = ax - cb.x, dy = ay - cb.y;
            // projections of d on the normals (cos_i, sin_i), (-sin_i, cos_i), then piece j's
            const float p0 = dx * ci + dy * si, p1 = dy * ci - dx * si;
            const float p2 = dx * cj + dy * sj, p3 = dy * cj - dx * sj;
            const float a0 = fabsf(p0), a1 = fabsf(p1), a2 = fabsf(p2), a3 = fabsf(p3);
            const float mx = fmaxf(fmaxf(a0, a1), fmaxf(a2, a3));
            const float pen = R - mx;
            if (!(take && pen > 0.f)) continue;
            cost += w * phi(phase, pen);
            viol = fmaxf(viol, pen);
            if (GRAD) {
                const float sc = w * dphi(phase, pen);
                {  // piece i: its own normals first (the first largest |projection|)
                    int best = 0;
                    float bm = a0;
                    if (a1 > bm) { bm = a1; best = 1; }
                    if (a2 > bm) { bm = a2; best = 2; }
                    if (a3 > bm) { best = 3; }
                    float nx, ny, pc, dn;
                    if (best == 0) { nx = ci; ny = si; pc = p0; dn = p1; }
                    else if (best == 1) { nx = -si; ny = ci; pc = p1; dn = -p0; }
                    else if (best == 2) { nx = cj; ny = sj; pc = p2; dn = 0.f; }
                    else { nx = -sj; ny = cj; pc = p3; dn = 0.f; }
                    const float sg = sgnf(pc);
                    g[0] -= sc * sg * nx;
                    g[1] -= sc * sg * ny;
                    g[3] += sc * (dR - sg * (dax * nx + day * ny + dn));
                }
                {  // piece j, as its own lane sees the pair: d -> -d, its normals first
                    int best = 2;
                    float bm = a2;
                    if (a3 > bm) { bm = a3; best = 3; }
                    if (a0 > bm) { bm = a0; best = 0; }
                    if (a1 > bm) { best = 1; }
                    float nx, ny, pc, dn;
                    if (best == 2) { nx = cj; ny = sj; pc = -p2; dn = -p3; }
                    else if (best == 3) { nx = -sj; ny = cj; pc = -p3; dn = p2; }
                    else if (best == 0) { nx = ci; ny = si; pc = -p0; dn = 0.f; }
                    else { nx = -si; ny = ci; pc = -p1; dn = 0.f; }
                    const float sg = sgnf(pc);
                    h0 -= sc * sg * nx;
                    h1 -= sc * sg * ny;
                    h3 += sc * (dRj - sg * (cb.z * nx + cb.w * ny + dn));
                }
            }
        }
        if (GRAD) {
            for (int d = 1; d < L; d <<= 1) {
                h0 += __shfl_xor(h0, d, 64);
                h1 += __shfl_xor(h1, d, 64);
                h3 += __shfl_xor(h3, d, 64);
            }
            if (k == 0) {
                float *o = s_gj + (i * T + t - 1) * 3;
                o[0] = h0;
                o[1] = h1;
                o[2] = h3;
            }
        }
    }
    if (GRAD) {
        __syncthreads();
        if (k == 0) {
            for (int t = 1; t <= T; ++t) {
                int src = i - t;
                if (src < 0) src += B;
                const float *o = s_gj + (src * T + t - 1) * 3;
                g[0] += o[0];
                g[1] += o[1];
                g[3] += o[2];
            }
        }
    }
}

// Stage-1 placement cost of one lane: the packing cost for packing problems, the tower /
// fixed-goal cost otherwise (the mode is uniform, so the branch does not diverge).
template <bool GRAD>
__device__ __forceinline__ void stage1_lane(const KProb &P, int phase, int i, int k, int L, const float *st,
                                            float4 *s_cell, float *s_gj, float &cost, float &viol, float (&g)[4])
{
    if (P.mode == SPASM_MODE_PACK)
        pack_particle<GRAD>(P, phase, i, k, L, st, s_cell, s_gj, cost, viol, g);
    else
        place_lane<GRAD>(P, phase, i, k, st, cost, viol, g);
}

// ------------------------------------------------------------------------------------
// Stage 1: sampling, placement cost/gradient and the gradient-descent loop.
// ------------------------------------------------------------------------------------
__global__ void k_sample(KProb P, int N, uint64_t seed, int round, float *x, const int *skip)
{
    if (skip && *skip) return;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= N * P.B) return;
    const int n = gid / P.B, i = gid % P.B;
    float u[4];
    uniforms4(seed, (uint64_t)n, (uint64_t)i, (uint64_t)round, 1u, u);
    float *o = x + (size_t)gid * 3;
    o[0] = P.samp_x0 + P.samp_xs * u[0];
    o[1] = P.samp_y0 + P.samp_ys * u[1];
    o[2] = -3.14159265358979f + 6.28318530717959f * u[2];
    if (P.yaw_steps > 0) {
        // yaw on yaw_steps directions; the step index is integer arithmetic on the 24-bit
        // draw, so no rounding can move a sample to a neighbouring direction
        const int k24 = (int)(u[2] * 16777216.0f);
        const int j = (int)(((long long)P.yaw_steps * k24) >> 24);
        o[2] = -3.14159265358979f + (6.28318530717959f / (float)P.yaw_steps) * (float)j;
    }
}

// One workgroup holds lcm(L B, 64) lanes = several particles, L = 2^lpb_log2 lanes per
// block (8 block spheres; for packing, the cells of the largest piece rounded up to a
// power of two, at least 4); lane = (particle, block, sphere or cell).  Steps k_begin..k_end-1 of
// descent (clamped to the region), then one evaluation at eval_phase.  Dynamic LDS:
// per particle and block 8 floats of state and 2 of reduction (and for packing the cell
// table and the pair gradients of pack_particle).
__global__ __launch_bounds__(1024) void k_place(KProb P, int n, const float *x_in, const int32_t *idx,
                                                float *x_out, int k_begin, int k_end, int eval_phase,
                                                float *cost_out, float *viol_out, float *gx_out, const int *skip)
{
    extern __shared__ float4 s_place4[];
    if (skip && *skip) return;
    const int B = P.B, lg = P.lpb_log2, L = 1 << lg, per = L * B, ppw = blockDim.x / per;
    const int tid = threadIdx.x, lp = tid / per, rem = tid % per, i = rem >> lg, k = rem & (L - 1);
    const bool pack = P.mode == SPASM_MODE_PACK;
    const int T = B >> 1;
    float4 *s_cell = s_place4;                                     // packing: [ppw][B L] cells
    float *s_state = (float *)(s_place4 + (pack ? ppw * B * L : 0));  // [ppw * B][8]
    float(*s_red)[2] = (float(*)[2])(s_state + ppw * B * 8);       // [ppw * B][2]
    float *s_gj = s_state + ppw * B * 10;                          // packing: [ppw][B][T][3]
    float4 *cell_p = s_cell + lp * B * L;
    float *gj_p = s_gj + lp * B * T * 3;
    const int p = blockIdx.x * ppw + lp;
    const bool valid = p < n;
    float *st = s_state + lp * B * 8;
    if (k == 0) {
        float x = 0.f, y = 0.f, yaw = 0.f;
        if (valid) {
            const int src = idx ? idx[p] : p;
            const float *xs = x_in + ((size_t)src * B + i) * 3;
            x = xs[0];
            y = xs[1];
            yaw = xs[2];
        }
        float s, c;
        sincosf(yaw, &s, &c);
        st[i * 8 + 0] = x;
        st[i * 8 + 1] = y;
        st[i * 8 + 2] = zstar(P, i);
        st[i * 8 + 3] = yaw;
        st[i * 8 + 4] = c;
        st[i * 8 + 5] = s;
    }
    __syncthreads();
    for (int kk = k_begin; kk < k_end; ++kk) {
        int phase;
        float lr;
        schedule(kk, P.k_lin1, P.eta1, P.alpha1, phase, lr);
        float c = 0.f, v = 0.f, g[4] = {0.f, 0.f, 0.f, 0.f};
        stage1_lane<true>(P, phase, i, k, L, st, cell_p, gj_p, c, v, g);
        for (int m = 1; m < L; m <<= 1) {
            g[0] += __shfl_xor(g[0], m, 64);
            g[1] += __shfl_xor(g[1], m, 64);
            g[3] += __shfl_xor(g[3], m, 64);
        }
        __syncthreads();
        if (k == 0) {
            const float x = fminf(fmaxf(st[i * 8 + 0] - lr * g[0], P.clamp_xl), P.clamp_xh);
            const float y = fminf(fmaxf(st[i * 8 + 1] - lr * g[1], P.clamp_yl), P.clamp_yh);
            const float yaw = st[i * 8 + 3] - lr * g[3];
            float s, cc;
            sincosf(yaw, &s, &cc);
            st[i * 8 + 0] = x;
            st[i * 8 + 1] = y;
            st[i * 8 + 3] = yaw;
            st[i * 8 + 4] = cc;
            st[i * 8 + 5] = s;
        }
        __syncthreads();
    }
    float c = 0.f, v = 0.f, g[4] = {0.f, 0.f, 0.f, 0.f};
    if (gx_out)
        stage1_lane<true>(P, eval_phase, i, k, L, st, cell_p, gj_p, c, v, g);
    else
        stage1_lane<false>(P, eval_phase, i, k, L, st, cell_p, gj_p, c, v, g);
    for (int m = 1; m < L; m <<= 1) {
        c += __shfl_xor(c, m, 64);
        v = fmaxf(v, __shfl_xor(v, m, 64));
        g[0] += __shfl_xor(g[0], m, 64);
        g[1] += __shfl_xor(g[1], m, 64);
        g[3] += __shfl_xor(g[3], m, 64);
    }
    if (k == 0) {
        s_red[lp * B + i][0] = c;
        s_red[lp * B + i][1] = v;
    }
    __syncthreads();
    if (!valid) return;
    if (k == 0) {
        if (gx_out) {
            float *o = gx_out + ((size_t)p * B + i) * 3;
            o[0] = g[0];
            o[1] = g[1];
            o[2] = g[3];
        }
        if (x_out) {
            float *o = x_out + ((size_t)p * B + i) * 3;
            o[0] = st[i * 8 + 0];
            o[1] = st[i * 8 + 1];
            o[2] = st[i * 8 + 3];
        }
        if (i == 0) {
            float cs = 0.f, vs = 0.f;
            for (int j = 0; j < B; ++j) {
                cs += s_red[lp * B + j][0];
                vs = fmaxf(vs, s_red[lp * B + j][1]);
            }
            if (cost_out) cost_out[p] = cs;
            if (viol_out) viol_out[p] = vs;
        }
    }
}

// ------------------------------------------------------------------------------------
// Stage 2: one particle per workgroup, one waypoint slot per lane.
// ------------------------------------------------------------------------------------
struct Slot {
    int s, w, b, tau;
    bool active;
};

// Joint axis screw of joint j+1 from frame T_j: xi = (z_j, o_j x z_j).  For a wrench
// (torque about the world origin t, force f) applied on links > j, <xi, (t, f)> is its
// contribution to dC/dq_{j+1}.
__device__ __forceinline__ float screw_dot(const Frame &F, const float (&wr)[6])
{
    const float m0 = F.p1 * F.z2 - F.p2 * F.z1, m1 = F.p2 * F.z0 - F.p0 * F.z2, m2 = F.p0 * F.z1 - F.p1 * F.z0;
    return F.z0 * wr[0] + F.z1 * wr[1] + F.z2 * wr[2] + m0 * wr[3] + m1 * wr[4] + m2 * wr[5];
}

// Forward pass over the links, fully unrolled so that every per-joint value is a
// register.  wr is the running wrench of all contacts on links < J+1 (torque about the
// origin, force); before link J+1's contacts are added, <xi_{J+1}, wr> is subtracted
// from g[J].  After the pass, g[j] + <xi_{j+1}, total wrench> is the reverse-mode
// gradient sum over links >= j+1 (second pass in slot_eval).
template <int J, bool GRAD, int CH, bool HB>
__device__ __forceinline__ void links_forward(const KProb &P, int phase, const Slot &sl, bool own_vis,
                                              const float (&q)[NJ], const float *s_pose, float *s_pacc, Frame &F,
                                              float &cost, float &viol, float (&g)[NJ], float (&wr)[6])
{
    if (GRAD) {
        // evaluate here: sinking it would keep every joint's axis and wrench live
        float t = screw_dot(F, wr);
        asm("" : "+v"(t));
        g[J] -= t;
    }
    dh_step(F, P.a[J], P.d[J], P.ca[J], P.sa[J], q[J]);
    float wt[3] = {wr[0], wr[1], wr[2]}, wf[3] = {wr[3], wr[4], wr[5]};
    for (int s0 = P.link_start[J]; s0 < P.link_start[J + 1]; s0 += CH) {
        float cx[CH], cy[CH], cz[CH], r[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const float4 sp = ldc(P.sph, s0 + i);
            cx[i] = F.p0 + sp.x * F.x0 + sp.y * F.y0 + sp.z * F.z0;
            cy[i] = F.p1 + sp.x * F.x1 + sp.y * F.y1 + sp.z * F.z1;
            cz[i] = F.p2 + sp.x * F.x2 + sp.y * F.y2 + sp.z * F.z2;
            r[i] = sp.w;
        }
        const LaneBox lb = lane_box<CH>(cx, cy, cz, r, sl.active);
        collide_boxes<GRAD, CH, HB>(P, phase, P.w[W_ARM], cx, cy, cz, r, lb, sl.active, cost, viol, wf, wt);
        if (P.mode != SPASM_MODE_P2P)  // a point-to-point problem has no blocks
            collide_blocks<GRAD, CH>(P, phase, P.w[W_ARM], cx, cy, cz, r, lb, sl.active, sl.b, own_vis, s_pose,
                                     s_pacc, cost, viol, wf, wt);
    }
    wr[0] = wt[0]; wr[1] = wt[1]; wr[2] = wt[2];
    wr[3] = wf[0]; wr[4] = wf[1]; wr[5] = wf[2];
    if constexpr (J + 1 < NJ)
        links_forward<J + 1, GRAD, CH, HB>(P, phase, sl, own_vis, q, s_pose, s_pacc, F, cost, viol, g, wr);
}

template <int J>
__device__ __forceinline__ void links_reverse(const KProb &P, const float (&q)[NJ], Frame &F, float (&g)[NJ],
                                              const float (&wr)[6])
{
    g[J] += screw_dot(F, wr);
    if constexpr (J + 1 < NJ) {
        dh_step(F, P.a[J], P.d[J], P.ca[J], P.sa[J], q[J]);
        links_reverse<J + 1>(P, q, F, g, wr);
    }
}

// Augmented-Lagrangian multipliers of one particle: lam [B][15] (nullable: plain
// penalties) for each block's grasp residual (components 0..5) and tie residual (6..14);
// with update set, the lanes that evaluate a residual also take the multiplier step
// lam += rho 2w e with it (the next evaluation sees the new values).
struct AlState {
    float *lam;
    bool update;
    float rho;
};

// Cost (and gradient) of one slot: arm spheres vs obstacles and blocks, held block,
// grasp alignment, tie to the placement, joint limits.  Smoothness and the placement
// cost are added by the caller.  GRAD: g[7] receives dC/dq of this slot, the pose
// gradient goes to the wave's LDS accumulator (arm/held contacts with placed blocks)
// and to s_tiepose (tie term).
template <bool GRAD, int CH, bool HB>
__device__ __forceinline__ void slot_eval(const KProb &P, int phase, const Slot &sl, int W, const float (&q)[NJ],
                                          const float *s_pose, float *s_pacc, float *s_tiepose, float &cost,
                                          float &viol, float (&g)[NJ], const AlState &al)
{
    const bool own_vis = sl.tau == 0 && sl.w < W - 1;
    float wr[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    Frame F;
    frame_identity(F);
    links_forward<0, GRAD, CH, HB>(P, phase, sl, own_vis, q, s_pose, s_pacc, F, cost, viol, g, wr);
    float et[3] = {wr[0], wr[1], wr[2]}, ef[3] = {wr[3], wr[4], wr[5]};
    // end effector and the block frame T_B = T_E G^-1
    const float pe0 = F.p0 + P.tool_d * F.z0, pe1 = F.p1 + P.tool_d * F.z1, pe2 = F.p2 + P.tool_d * F.z2;
    const float *Gr = P.Gi_R;
    // column c of R_B = R_E * (Gr[0][c], Gr[1][c], Gr[2][c])
    float RB[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        RB[0][c] = Gr[c] * F.x0 + Gr[3 + c] * F.y0 + Gr[6 + c] * F.z0;
        RB[1][c] = Gr[c] * F.x1 + Gr[3 + c] * F.y1 + Gr[6 + c] * F.z1;
        RB[2][c] = Gr[c] * F.x2 + Gr[3 + c] * F.y2 + Gr[6 + c] * F.z2;
    }
    const float tb0 = pe0 + P.Gi_t[0] * F.x0 + P.Gi_t[1] * F.y0 + P.Gi_t[2] * F.z0;
    const float tb1 = pe1 + P.Gi_t[0] * F.x1 + P.Gi_t[1] * F.y1 + P.Gi_t[2] * F.z1;
    const float tb2 = pe2 + P.Gi_t[0] * F.x2 + P.Gi_t[1] * F.y2 + P.Gi_t[2] * F.z2;

    // held block (Appendix B C_block, interior transfer waypoints)
    const bool held = sl.active && sl.tau == 1 && sl.w >= 1 && sl.w <= W - 2;
    if (__any(held)) {
        const float so = P.sph_off, rb = P.r_blk;
        float cx[8], cy[8], cz[8], r[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float s0 = (k & 1) ? so : -so, s1 = (k & 2) ? so : -so, s2 = (k & 4) ? so : -so;
            cx[k] = tb0 + RB[0][0] * s0 + RB[0][1] * s1 + RB[0][2] * s2;
            cy[k] = tb1 + RB[1][0] * s0 + RB[1][1] * s1 + RB[1][2] * s2;
            cz[k] = tb2 + RB[2][0] * s0 + RB[2][1] * s1 + RB[2][2] * s2;
            r[k] = rb;
        }
        const float w_block = P.w[W_BLOCK];
        // bounds of the eight spheres: centre +- (so * row sums of |R_B| + rb)
        LaneBox lb{INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        if (held) {
            const float e0 = so * (fabsf(RB[0][0]) + fabsf(RB[0][1]) + fabsf(RB[0][2])) + rb + 1e-4f;
            const float e1 = so * (fabsf(RB[1][0]) + fabsf(RB[1][1]) + fabsf(RB[1][2])) + rb + 1e-4f;
            const float e2 = so * (fabsf(RB[2][0]) + fabsf(RB[2][1]) + fabsf(RB[2][2])) + rb + 1e-4f;
            lb = LaneBox{tb0 - e0, tb1 - e1, tb2 - e2, tb0 + e0, tb1 + e1, tb2 + e2};
        }
        collide_boxes<GRAD, 8>(P, phase, w_block, cx, cy, cz, r, lb, held, cost, viol, ef, et);
        collide_blocks<GRAD, 8>(P, phase, w_block, cx, cy, cz, r, lb, held, sl.b, false, s_pose, s_pacc, cost,
                                viol, ef, et);
    }
    // grasp alignment at the first transfer waypoint (C_start: position, roll/pitch)
    if (sl.active && sl.tau == 1 && sl.w == 0) {
        const float w_st = P.w[W_START];
        const float4 I = ldc(P.blk_init, 2 * sl.b);
        const float rp0 = tb0 - I.x, rp1 = tb1 - I.y, rp2 = tb2 - I.z;
        const float u0 = RB[0][2], u1 = RB[1][2], u2 = RB[2][2];
        const float rz0 = u0, rz1 = u1, rz2 = u2 - 1.f;
        const float c2 = rp0 * rp0 + rp1 * rp1 + rp2 * rp2 + rz0 * rz0 + rz1 * rz1 + rz2 * rz2;
        cost += w_st * c2;
        viol = fmaxf(viol, sqrtf(c2));
        float l[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (al.lam) {
            float *lb = al.lam + 15 * sl.b;
            const float e[6] = {rp0, rp1, rp2, rz0, rz1, rz2};
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                l[c] = lb[c];
                cost += l[c] * e[c];
                if (al.update) lb[c] = l[c] + al.rho * 2.f * w_st * e[c];
            }
        }
        if (GRAD) {
            const float f0 = 2.f * w_st * rp0 + l[0], f1 = 2.f * w_st * rp1 + l[1], f2 = 2.f * w_st * rp2 + l[2];
            const float h0 = 2.f * w_st * rz0 + l[3], h1 = 2.f * w_st * rz1 + l[4], h2 = 2.f * w_st * rz2 + l[5];
            ef[0] += f0;
            ef[1] += f1;
            ef[2] += f2;
            et[0] += tb1 * f2 - tb2 * f1 + u1 * h2 - u2 * h1;
            et[1] += tb2 * f0 - tb0 * f2 + u2 * h0 - u0 * h2;
            et[2] += tb0 * f1 - tb1 * f0 + u0 * h1 - u1 * h0;
        }
    }
    // tie of the carried block to its placement variable at the last transfer waypoint
    if (sl.active && sl.tau == 1 && sl.w == W - 1) {
        const float w_t = P.w[W_TIE];
        const float *pp = s_pose + sl.b * 8;
        const float cps = pp[4], sps = pp[5];
        const float rp0 = tb0 - pp[0], rp1 = tb1 - pp[1], rp2 = tb2 - pp[2];
        const float ux0 = RB[0][0], ux1 = RB[1][0], ux2 = RB[2][0];
        const float uz0 = RB[0][2], uz1 = RB[1][2], uz2 = RB[2][2];
        const float rx0 = ux0 - cps, rx1 = ux1 - sps, rx2 = ux2;
        const float rz0 = uz0, rz1 = uz1, rz2 = uz2 - 1.f;
        const float c2 = rp0 * rp0 + rp1 * rp1 + rp2 * rp2 + rx0 * rx0 + rx1 * rx1 + rx2 * rx2 + rz0 * rz0 +
                         rz1 * rz1 + rz2 * rz2;
        cost += w_t * c2;
        viol = fmaxf(viol, sqrtf(c2));
        float l[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (al.lam) {
            float *lb = al.lam + 15 * sl.b + 6;
            const float e[9] = {rp0, rp1, rp2, rx0, rx1, rx2, rz0, rz1, rz2};
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                l[c] = lb[c];
                cost += l[c] * e[c];
                if (al.update) lb[c] = l[c] + al.rho * 2.f * w_t * e[c];
            }
        }
        if (GRAD) {
            const float f0 = 2.f * w_t * rp0 + l[0], f1 = 2.f * w_t * rp1 + l[1], f2 = 2.f * w_t * rp2 + l[2];
            const float hx0 = 2.f * w_t * rx0 + l[3], hx1 = 2.f * w_t * rx1 + l[4], hx2 = 2.f * w_t * rx2 + l[5];
            const float hz0 = 2.f * w_t * rz0 + l[6], hz1 = 2.f * w_t * rz1 + l[7], hz2 = 2.f * w_t * rz2 + l[8];
            ef[0] += f0;
            ef[1] += f1;
            ef[2] += f2;
            et[0] += tb1 * f2 - tb2 * f1 + ux1 * hx2 - ux2 * hx1 + uz1 * hz2 - uz2 * hz1;
            et[1] += tb2 * f0 - tb0 * f2 + ux2 * hx0 - ux0 * hx2 + uz2 * hz0 - uz0 * hz2;
            et[2] += tb0 * f1 - tb1 * f0 + ux0 * hx1 - ux1 * hx0 + uz0 * hz1 - uz1 * hz0;
            float *tp = s_tiepose + sl.b * 4;
            tp[0] = -f0;
            tp[1] = -f1;
            tp[2] = -f2;
            tp[3] = -(hx0 * -sps + hx1 * cps);
        }
    }
    if (GRAD) {
        const float wtot[6] = {et[0], et[1], et[2], ef[0], ef[1], ef[2]};
        // Recompute the frames rather than keep all seven live across the contact loops;
        // the opaque copy stops the compiler from merging the two passes.
        float qr[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            qr[j] = q[j];
            asm("" : "+v"(qr[j]));
        }
        frame_identity(F);
        links_reverse<0>(P, qr, F, g, wtot);
    }
    // joint-limit hinges
    if (sl.active) {
        const float w_l = P.w[W_LIM];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const float eh = q[j] - P.hi[j], el = P.lo[j] - q[j];
            if (eh > 0.f) {
                cost += w_l * phi(phase, eh);
                viol = fmaxf(viol, eh);
                if (GRAD) g[j] += w_l * dphi(phase, eh);
            }
            if (el > 0.f) {
                cost += w_l * phi(phase, el);
                viol = fmaxf(viol, el);
                if (GRAD) g[j] -= w_l * dphi(phase, el);
            }
        }
    }
}

// Whole-particle evaluation shared by every stage-2 mode: slot terms, smoothness (lane
// shuffles: a segment is W consecutive lanes inside one wave) and the placement cost of
// the pose variables (lanes tid < 8B, one block sphere each).
template <bool GRAD, int CH, bool HB = false>
__device__ __forceinline__ void particle_eval(const KProb &P, int phase, const Slot &sl, int W, const float (&q)[NJ],
                                              const float *s_pose, float *s_pacc_wave, float *s_tiepose,
                                              float *s_placeg, float &cost, float &viol, float (&g)[NJ], const AlState &al)
{
    slot_eval<GRAD, CH, HB>(P, phase, sl, W, q, s_pose, s_pacc_wave, s_tiepose, cost, viol, g, al);
    const float w_s = P.w[W_SMOOTH];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const float qn = lane_next(q[j]);
        const float qp = lane_prev(q[j]);
        if (sl.active && sl.w < W - 1) {
            const float d = qn - q[j];
            cost += w_s * d * d;
            if (GRAD) g[j] -= 2.f * w_s * d;
        }
        if (GRAD && sl.active && sl.w > 0) g[j] += 2.f * w_s * (q[j] - qp);
    }
    const int tid = threadIdx.x;
    if (tid < 8 * MAX_B) {
        const int i = tid >> 3, k = tid & 7;
        float gp[4] = {0.f, 0.f, 0.f, 0.f};
        if (i < P.B && P.mode != SPASM_MODE_P2P) place_lane<GRAD>(P, phase, i, k, s_pose, cost, viol, gp);
        if (GRAD) {
#pragma unroll
            for (int c = 0; c < 4; ++c) gp[c] = group8_reduce(gp[c], OpSum());
            if (k == 0 && i < P.B) {
                s_placeg[i * 4 + 0] = gp[0];
                s_placeg[i * 4 + 1] = gp[1];
                s_placeg[i * 4 + 2] = gp[2];
                s_placeg[i * 4 + 3] = gp[3];
            }
        }
    }
}

// Pose table entry: x, y, z, yaw, cos, sin, and the xy half extent of the yawed square.
__device__ __forceinline__ void set_pose_entry(float *s_pose, int b, float x, float y, float z, float yaw, float half)
{
    float s, c;
    sincosf(yaw, &s, &c);
    float *pp = s_pose + b * 8;
    pp[0] = x;
    pp[1] = y;
    pp[2] = z;
    pp[3] = yaw;
    pp[4] = c;
    pp[5] = s;
    pp[6] = half * (fabsf(c) + fabsf(s));
}

// Adam (torch semantics): step = lr / (1 - b1^k), ibc2 = 1 / sqrt(1 - b2^k); the square
// root and reciprocal use the hardware instructions (about 1 ulp).
__device__ __forceinline__ float adam_update(float x, float &m, float &v, float g, float step, float b1, float b2,
                                             float eps, float ibc2)
{
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    return x - step * m * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v) * ibc2 + eps);
}

// One particle per workgroup.  MODE 0: cost, 1: cost + gradient (optionally scaled per
// particle), 2: optimise.  s_mv: dynamic LDS, [2][NJ][blockDim.x] Adam moments (MODE 2).
// HB: the obstacle broad phase bounds each half wave (the optimisation launches).  FINE: a
// particle of 9-12 waves with a CU to itself (the 768-thread launches) takes the finer
// issue-priority step.
template <int MODE, int CH, bool HB = false, bool FINE = false>
__device__ __forceinline__ void traj_particle(const KProb &P, const TrajArgs &a, int p, float *s_mv)
{
    __shared__ float s_pose[2 * MAX_B * 8];
    __shared__ float s_pacc[16 * MAX_B * 4];
    __shared__ float s_tiepose[MAX_B * 4];
    __shared__ float s_placeg[MAX_B * 4];
    __shared__ float s_tie[2][2 * MAX_B][8];
    __shared__ float s_red[16][2];
    __shared__ float s_popt[2][MAX_B * 4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    // lanes [0, BW) are the transit segments (the single motion of a p2p problem, B = 1)
    const int B = P.B, W = a.W, NS = n_segments(P), BW = B * W;
    Slot sl;
    sl.active = tid < NS * W;
    if (tid < BW) {
        sl.s = 2 * (tid / W);
        sl.w = tid % W;
    } else if (sl.active) {
        const int t2 = tid - BW;
        sl.s = 2 * (t2 / W) + 1;
        sl.w = t2 % W;
    } else {
        sl.s = 0;
        sl.w = 0;
    }
    sl.b = sl.s >> 1;
    sl.tau = sl.s & 1;
    const size_t qoff = (((size_t)p * NS + sl.s) * W + sl.w) * NJ;
    float q[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] = sl.active ? a.q_in[qoff + j] : 0.f;
    if (tid < B) {
        if (a.pose_in) {
            const float *pi = a.pose_in + ((size_t)p * B + tid) * 4;
            set_pose_entry(s_pose, tid, pi[0], pi[1], pi[2], pi[3], P.half);
        } else {  // p2p problems take no poses
            set_pose_entry(s_pose, tid, 0.f, 0.f, 0.f, 0.f, P.half);
        }
    } else if (tid < 2 * B) {  // blockDim >= 64 >= 2 * MAX_B
        const int b = tid - B;
        const float4 a0 = ldc(P.blk_init, 2 * b), a1 = ldc(P.blk_init, 2 * b + 1);
        float *pp = s_pose + (MAX_B + b) * 8;
        pp[0] = a0.x;
        pp[1] = a0.y;
        pp[2] = a0.z;
        pp[3] = a0.w;
        pp[4] = a1.x;
        pp[5] = a1.y;
        pp[6] = P.half * (fabsf(a1.x) + fabsf(a1.y));
    }
    float *s_pacc_w = s_pacc + wave * MAX_B * 4;
    if (lane < 4 * B) s_pacc_w[lane] = 0.f;
    // each block's tie lane rewrites its entry on every evaluation; a problem without
    // transfer segments (point to point) never does, so it must read zeros
    if (tid < 4 * B) s_tiepose[tid] = 0.f;
    const size_t per_opt = (size_t)2 * BW * NJ + 4 * B;
    const size_t ostride = a.opt_stride ? (size_t)a.opt_stride : 2 * per_opt;  // floats per particle in opt
    AlState al{a.lam ? a.lam + (size_t)p * a.lam_stride : nullptr, false, P.al_rho};
    if (MODE == 2) {
        const float *om = a.opt ? a.opt + (size_t)p * ostride : nullptr;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            s_mv[(0 * NJ + j) * blockDim.x + tid] = (om && sl.active) ? om[(sl.s * W + sl.w) * NJ + j] : 0.f;
            s_mv[(1 * NJ + j) * blockDim.x + tid] =
                (om && sl.active) ? om[per_opt + (sl.s * W + sl.w) * NJ + j] : 0.f;
        }
        if (tid < 4 * B) {
            s_popt[0][tid] = om ? om[2 * BW * NJ + tid] : 0.f;
            s_popt[1][tid] = om ? om[per_opt + 2 * BW * NJ + tid] : 0.f;
        }
    }
    __syncthreads();

    if (lane == 0) s_wave_work[wave] = 0;
    if (MODE == 2) {
        const float b1 = P.beta1, b2 = P.beta2, eps = P.adam_eps;
        for (int k = a.k_begin; k < a.k_end; ++k) {
            {
                // issue priority from the previous iteration's contact work: the waves
                // that hold their particles back run first on their SIMDs (scheduling
                // only; the arithmetic is the same)
                const int lvl = __builtin_amdgcn_readfirstlane(s_wave_work[wave]) / (FINE ? PRIO_STEP_HB : PRIO_STEP);
                if (lane == 0) s_wave_work[wave] = 0;
                if (lvl >= 3)
                    __builtin_amdgcn_s_setprio(3);
                else if (lvl == 2)
                    __builtin_amdgcn_s_setprio(2);
                else if (lvl == 1)
                    __builtin_amdgcn_s_setprio(1);
                else
                    __builtin_amdgcn_s_setprio(0);
            }
            int phase;
            float lr;
            schedule(k, a.k_lin2, P.eta2, P.alpha2, phase, lr);
            float cost = 0.f, viol = 0.f, g[NJ] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            al.update = al.lam && P.al_every > 0 && k % P.al_every == 0;
            particle_eval<true, CH, HB>(P, phase, sl, W, q, s_pose, s_pacc_w, s_tiepose, s_placeg, cost, viol, g,
                                        al);
            if (sl.active && sl.w == W - 1)
                for (int j = 0; j < NJ; ++j) s_tie[0][sl.s][j] = g[j];
            if (sl.active && sl.w == 0)
                for (int j = 0; j < NJ; ++j) s_tie[1][sl.s][j] = g[j];
            __syncthreads();
            const float bc1 = 1.f - powf(b1, (float)k), bc2s = sqrtf(1.f - powf(b2, (float)k));
            const float step = lr / bc1, ibc2 = 1.f / bc2s;
            // the start configuration (first waypoint of the first segment) is pinned
            // at q_home in every mode, and so is the goal of a point-to-point motion
            if (sl.active && !(sl.s == 0 && sl.w == 0) && !(P.mode == SPASM_MODE_P2P && sl.w == W - 1)) {
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    float gj = g[j];
                    if (sl.w == W - 1 && sl.s + 1 < NS) gj = g[j] + s_tie[1][sl.s + 1][j];
                    if (sl.w == 0 && sl.s > 0) gj = s_tie[0][sl.s - 1][j] + g[j];
                    float &m = s_mv[(0 * NJ + j) * blockDim.x + tid];
                    float &v = s_mv[(1 * NJ + j) * blockDim.x + tid];
                    float mm = m, vv = v;
                    q[j] = adam_update(q[j], mm, vv, gj, step, b1, b2, eps, ibc2);
                    m = mm;
                    v = vv;
                }
            }
            if (P.mode == 0 && tid < 4 * B) {
                const int bb = tid >> 2, c = tid & 3;
                float gsum = 0.f;
                for (int wv = 0; wv < nwave; ++wv) gsum += s_pacc[(wv * MAX_B + bb) * 4 + c];
                gsum += s_placeg[bb * 4 + c];
                gsum += s_tiepose[bb * 4 + c];
                float mm = s_popt[0][tid], vv = s_popt[1][tid];
                const float x = adam_update(s_pose[bb * 8 + c], mm, vv, gsum, step, b1, b2, eps, ibc2);
                s_popt[0][tid] = mm;
                s_popt[1][tid] = vv;
                s_pose[bb * 8 + c] = x;
                if (c == 3) {
                    float s, cc;
                    sincosf(x, &s, &cc);
                    s_pose[bb * 8 + 4] = cc;
                    s_pose[bb * 8 + 5] = s;
                    s_pose[bb * 8 + 6] = P.half * (fabsf(cc) + fabsf(s));
                }
            }
            __syncthreads();
            if (lane < 4 * B) s_pacc_w[lane] = 0.f;
        }
        // write the state back, then evaluate the final state (quadratic phase)
        if (sl.active) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) a.q_out[qoff + j] = q[j];
        }
        if (tid < 4 * B && a.pose_out) {
            const int bb = tid >> 2, c = tid & 3;
            a.pose_out[((size_t)p * B + bb) * 4 + c] = s_pose[bb * 8 + c];
        }
        if (a.opt) {
            float *om = a.opt + (size_t)p * ostride;
            if (sl.active)
                for (int j = 0; j < NJ; ++j) {
                    om[(sl.s * W + sl.w) * NJ + j] = s_mv[(0 * NJ + j) * blockDim.x + tid];
                    om[per_opt + (sl.s * W + sl.w) * NJ + j] = s_mv[(1 * NJ + j) * blockDim.x + tid];
                }
            if (tid < 4 * B) {
                om[2 * BW * NJ + tid] = s_popt[0][tid];
                om[per_opt + 2 * BW * NJ + tid] = s_popt[1][tid];
            }
        }
        if (!a.cost && !a.viol) return;
        float cost = 0.f, viol = 0.f, g[NJ] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        // the final evaluation ranks particles by the plain cost (no multiplier terms)
        particle_eval<false, CH>(P, 1, sl, W, q, s_pose, s_pacc_w, s_tiepose, s_placeg, cost, viol, g,
                                 AlState{nullptr, false, 0.f});
        cost = wave_sum(cost);
        viol = wave_max(viol);
        if (lane == 0) {
            s_red[wave][0] = cost;
            s_red[wave][1] = viol;
        }
        __syncthreads();
        if (tid == 0) {
            float c = 0.f, v = 0.f;
            for (int wv = 0; wv < nwave; ++wv) {
                c += s_red[wv][0];
                v = fmaxf(v, s_red[wv][1]);
            }
            if (a.cost) a.cost[p] = c;
            if (a.viol) a.viol[p] = v;
        }
        return;
    }

    // MODE 0 / 1: one evaluation
    float cost = 0.f, viol = 0.f, g[NJ] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    particle_eval<MODE == 1, CH>(P, a.phase, sl, W, q, s_pose, s_pacc_w, s_tiepose, s_placeg, cost, viol, g, al);
    cost = wave_sum(cost);
    viol = wave_max(viol);
    if (lane == 0) {
        s_red[wave][0] = cost;
        s_red[wave][1] = viol;
    }
    __syncthreads();
    const float scale = a.gout ? a.gout[p] : 1.f;
    if (tid == 0) {
        float c = 0.f, v = 0.f;
        for (int wv = 0; wv < nwave; ++wv) {
            c += s_red[wv][0];
            v = fmaxf(v, s_red[wv][1]);
        }
        if (a.cost) a.cost[p] = c;
        if (a.viol) a.viol[p] = v;
    }
    if (MODE == 1) {
        if (sl.active && a.gq) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) a.gq[qoff + j] = g[j] * scale;
        }
        if (a.gpose && tid < 4 * B) {
            const int bb = tid >> 2, c = tid & 3;
            float gsum = 0.f;
            for (int wv = 0; wv < nwave; ++wv) gsum += s_pacc[(wv * MAX_B + bb) * 4 + c];
            gsum += s_placeg[bb * 4 + c];
            gsum += s_tiepose[bb * 4 + c];
            a.gpose[((size_t)p * B + bb) * 4 + c] = gsum * scale;
        }
    }
}

// BOUND: the launch bound the registers are allocated for -- 1024 threads (128 VGPRs, 16
// waves per CU) or 768 (168 VGPRs, 12 waves per CU; fewer spills).  The optimisation
// launch takes 768 when a CU holds as many of its particles either way (6 or 9-12 waves
// per particle, e.g. a 10-block tower: one particle per CU).  Every optimisation launch
// bounds each half wave (one segment of 32 waypoints) on its own in the obstacle broad
// phase.
template <int MODE, int CH, int BOUND = 1024>
__global__ __launch_bounds__(BOUND) void k_traj(KProb P, TrajArgs a)
{
    extern __shared__ float s_mv[];
    if (a.skip && __builtin_amdgcn_readfirstlane(*a.skip)) return;
    const int p = a.perm ? a.perm[a.P - 1 - (int)blockIdx.x] : (int)blockIdx.x;
    traj_particle<MODE, CH, MODE == 2, BOUND == 768>(P, a, p, s_mv);
}

// Serving: one launch advances every active solve of one (thread count, sphere chunk)
// class; workgroup w belongs to the last solve whose `first` is <= w.  Descriptors are
// read through the constant address space so that their fields stay in scalar registers.
typedef __attribute__((address_space(4))) const char cchar;

template <int CH, int BOUND>
__global__ __launch_bounds__(BOUND) void k_serve(const ServeSolve *solves, int nsolve)
{
    extern __shared__ float s_mv[];
    cchar *base = (cchar *)solves;
    const int wg = blockIdx.x;
    int lo = 0, hi = nsolve - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int first = *(const int *)(base + (size_t)mid * sizeof(ServeSolve) + offsetof(ServeSolve, first));
        if (first <= wg)
            lo = mid;
        else
            hi = mid - 1;
    }
    const ServeSolve &d = *(const ServeSolve *)(base + (size_t)lo * sizeof(ServeSolve));
    traj_particle<2, CH, true, BOUND == 768>(d.P, d.a, wg - d.first, s_mv);
}

// ------------------------------------------------------------------------------------
// Selection (ArgSort of Alg. 1) for up to 16384 unique 64-bit keys, by rank:
// kind 0 (top-M):  key = ordered(cost) << 32 | index
// kind 1 (order):  key = unsatisfied << 63 | cost bits << 32 | index   (cost >= 0)
// kind 2:          keys read from memory (the radix select's survivors)
// Keys are unique (the index is in them), so the sorted position of a key is the number
// of keys below it.  Every workgroup builds all n keys in LDS; workgroup g ranks keys
// [g KB, (g + 1) KB): thread t takes key g KB + (t mod KB) and compares it with one
// contiguous slice of the n keys; the partial counts are summed (lane shuffles, then
// LDS) and key i goes to slot rank(i) when that is below nout.  O(n^2) comparisons
// spread over n / KB workgroups: a few microseconds where one workgroup's sorting network
// would take tens.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ordered_bits(float f)
{
    if (f != f) f = __int_as_float(0x7f800000);
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(1024) void k_rank_sort(int kind, int n, int kb_log2, const float *cost, const float *viol,
                                                    float eps, const unsigned long long *in_keys, int nout,
                                                    int32_t *out_idx, int32_t *out_count, const int *skip)
{
    extern __shared__ unsigned long long s_keys[];  // n keys, then 16 x 64 partial counts
    __shared__ int s_cnt;
    if (skip && *skip) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int KB = 1 << kb_log2, NS = 1024 >> kb_log2;
    if (tid == 0) s_cnt = 0;
    int cnt = 0;
    for (int i = tid; i < n; i += 1024) {
        unsigned long long key;
        if (kind == 0) {
            key = ((unsigned long long)ordered_bits(cost[i]) << 32) | (unsigned)i;
        } else if (kind == 1) {
            float c = cost[i];
            if (c != c) c = __int_as_float(0x7f800000);
            c = fmaxf(c, 0.f);
            const bool unsat = !(viol[i] < eps);
            cnt += !unsat;
            key = ((unsigned long long)unsat << 63) | ((unsigned long long)(__float_as_uint(c) & 0x7fffffffu) << 32) |
                  (unsigned)i;
        } else {
            key = in_keys[i];
        }
        s_keys[i] = key;
    }
    __syncthreads();  // keys are in; s_cnt is cleared
    const int kb = tid & (KB - 1), sl = tid >> kb_log2;
    const int i = blockIdx.x * KB + kb;
    const unsigned long long ki = i < n ? s_keys[i] : ~0ull;
    const int len = (n + NS - 1) / NS, j0 = sl * len, j1 = min(n, j0 + len);
    uint32_t r = 0;
#pragma unroll 8
    for (int j = j0; j < j1; ++j) r += s_keys[j] < ki ? 1u : 0u;
    for (int d = KB; d < 64; d <<= 1) r += __shfl_xor(r, d, 64);
    uint32_t *s_part = (uint32_t *)(s_keys + n);
    if (lane < KB) s_part[wave * 64 + lane] = r;
    if (cnt) atomicAdd(&s_cnt, cnt);
    __syncthreads();
    if (tid < KB && i < n) {
        uint32_t rank = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) rank += s_part[w * 64 + tid];
        if (rank < (uint32_t)nout) out_idx[rank] = (int32_t)(ki & 0xffffffffu);
    }
    if (out_count && blockIdx.x == 0 && tid == 0) *out_count = kind == 1 ? s_cnt : nout;
}

// ------------------------------------------------------------------------------------
// Top-M beyond one workgroup's sort (Alg. 1 ArgSort[:M] for N up to 2^20): radix select.
// Three counting passes over the ordered 32-bit cost (digits of 11, 11 and 10 bits) find
// the value T of the M-th smallest key, the number of keys below it, and how many keys
// equal to T are still needed; the keys below T and the first of the keys equal to T in
// index order are collected (exactly the M smallest (cost, index) pairs) and sorted in
// one workgroup.  State in the workspace: prefix, mask, need, below.
// ------------------------------------------------------------------------------------
constexpr int RS_KEYS = 4096;  // keys per workgroup in the counting passes

__device__ __forceinline__ void rs_digit(int pass, int &shift, int &bins)
{
    shift = pass == 0 ? 21 : pass == 1 ? 10 : 0;
    bins = pass == 2 ? 1024 : 2048;
}

__global__ __launch_bounds__(1024) void k_rs_init(int M, uint32_t *state, uint32_t *hist)
{
    const int tid = threadIdx.x;
    if (tid == 0) {
        state[0] = 0;  // prefix: the bits of T fixed so far
        state[1] = 0;  // mask of those bits
        state[2] = (uint32_t)M;  // keys still needed among those matching the prefix
        state[3] = 0;  // keys known to lie below T
    }
    for (int i = tid; i < 2048; i += blockDim.x) hist[i] = 0;
}

__global__ __launch_bounds__(1024) void k_rs_hist(int n, const float *cost, int pass, const uint32_t *state,
                                                  uint32_t *hist)
{
    __shared__ uint32_t s_h[2048];
    int shift, bins;
    rs_digit(pass, shift, bins);
    const int tid = threadIdx.x;
    for (int i = tid; i < bins; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const uint32_t prefix = state[0], mask = state[1];
    const int lo = blockIdx.x * RS_KEYS, hi = min(n, lo + RS_KEYS);
    for (int e = lo + tid; e < hi; e += blockDim.x) {
        const uint32_t u = ordered_bits(cost[e]);
        if ((u & mask) == prefix) atomicAdd(&s_h[(u >> shift) & (uint32_t)(bins - 1)], 1u);
    }
    __syncthreads();
    for (int i = tid; i < bins; i += blockDim.x)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

// One workgroup of 1024 threads, two bins each: the bin in which the running count
// reaches need fixes the next digit of T; the histogram is cleared for the next pass.
__global__ __launch_bounds__(1024) void k_rs_pick(int pass, uint32_t *state, uint32_t *hist)
{
    __shared__ uint32_t s_w[16];
    int shift, bins;
    rs_digit(pass, shift, bins);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t h0 = 2 * tid < bins ? hist[2 * tid] : 0u, h1 = 2 * tid + 1 < bins ? hist[2 * tid + 1] : 0u;
    const uint32_t prefix = state[0], mask = state[1], need = state[2], below0 = state[3];
    uint32_t incl = h0 + h1;  // inclusive scan over the threads' pairs
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int w = 0; w < wave; ++w) off += s_w[w];
    incl += off;
    const uint32_t excl = incl - h0 - h1;
    int b = -1;
    uint32_t below = 0;
    if (excl < need && need <= excl + h0) {
        b = 2 * tid;
        below = excl;
    } else if (excl + h0 < need && need <= incl) {
        b = 2 * tid + 1;
        below = excl + h0;
    }
    __syncthreads();  // every thread has read the state and its bins
    if (b >= 0) {
        state[0] = prefix | ((uint32_t)b << shift);
        state[1] = mask | ((uint32_t)(bins - 1) << shift);
        state[2] = need - below;
        state[3] = below0 + below;
    }
    if (2 * tid < 2048) hist[2 * tid] = 0;
    if (2 * tid + 1 < 2048) hist[2 * tid + 1] = 0;
}

// Keys below T and keys equal to T per workgroup range.
__global__ __launch_bounds__(1024) void k_rs_count(int n, const float *cost, const uint32_t *state, uint32_t *wg_lt,
                                                   uint32_t *wg_eq)
{
    __shared__ uint32_t s_l[16], s_e[16];
    const uint32_t T = state[0];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lo = blockIdx.x * RS_KEYS, hi = min(n, lo + RS_KEYS);
    uint32_t cl = 0, ce = 0;
    for (int e = lo + tid; e < hi; e += blockDim.x) {
        const uint32_t u = ordered_bits(cost[e]);
        cl += u < T ? 1u : 0u;
        ce += u == T ? 1u : 0u;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        cl += __shfl_xor(cl, d, 64);
        ce += __shfl_xor(ce, d, 64);
    }
    if (lane == 0) {
        s_l[wave] = cl;
        s_e[wave] = ce;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t tl = 0, te = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            tl += s_l[w];
            te += s_e[w];
        }
        wg_lt[blockIdx.x] = tl;
        wg_eq[blockIdx.x] = te;
    }
}

// Collect the M keys without atomics: keys below T go to slots in index order (this
// workgroup's base is the count below T in the ranges before it), then the keys equal to
// T, after all keys below T, while their rank in index order is below need.
__global__ __launch_bounds__(1024) void k_rs_collect(int n, const float *cost, const uint32_t *state,
                                                     const uint32_t *wg_lt, const uint32_t *wg_eq, int M,
                                                     unsigned long long *surv)
{
    __shared__ uint32_t s_l[16], s_e[16];
    __shared__ uint32_t s_base[2];
    const uint32_t T = state[0], need = state[2], below = state[3];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    if (tid < 2) {
        const uint32_t *c = tid == 0 ? wg_lt : wg_eq;
        uint32_t b = 0;
        for (int g = 0; g < (int)blockIdx.x; ++g) b += c[g];
        s_base[tid] = b;
    }
    __syncthreads();
    uint32_t run_l = s_base[0], run_e = s_base[1];
    const int lo = blockIdx.x * RS_KEYS, hi = min(n, lo + RS_KEYS);
    const unsigned long long below_lane = (1ull << lane) - 1ull;
    for (int e0 = lo; e0 < hi; e0 += blockDim.x) {
        const int e = e0 + tid;
        uint32_t u = 0;
        bool lt = false, eq = false;
        if (e < hi) {
            u = ordered_bits(cost[e]);
            lt = u < T;
            eq = u == T;
        }
        const unsigned long long key = ((unsigned long long)u << 32) | (uint32_t)e;
        const unsigned long long bl = __ballot(lt), be = __ballot(eq);
        if (lane == 0) {
            s_l[wave] = (uint32_t)__popcll(bl);
            s_e[wave] = (uint32_t)__popcll(be);
        }
        __syncthreads();
        uint32_t before_l = 0, before_e = 0, total_l = 0, total_e = 0;
        for (int w = 0; w < nwave; ++w) {
            const uint32_t cl = s_l[w], ce = s_e[w];
            if (w < wave) {
                before_l += cl;
                before_e += ce;
            }
            total_l += cl;
            total_e += ce;
        }
        // slots stay below M by construction (below + need = M); the checks only guard it
        if (lt) {
            const uint32_t slot = run_l + before_l + (uint32_t)__popcll(bl & below_lane);
            if (slot < (uint32_t)M) surv[slot] = key;
        }
        if (eq) {
            const uint32_t r = run_e + before_e + (uint32_t)__popcll(be & below_lane);
            if (r < need && below + r < (uint32_t)M) surv[below + r] = key;
        }
        run_l += total_l;
        run_e += total_e;
        __syncthreads();  // s_l and s_e are rewritten next round
    }
}

// Placement round output: particles in satisfying-first order with their cost and
// violation.
__global__ void k_gather_place(int B, int M, const float *xs, const float *cs, const float *vs, const int32_t *ord,
                               float *x_out, float *c_out, float *v_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int src = ord[i];
    for (int k = 0; k < 3 * B; ++k) x_out[(size_t)i * 3 * B + k] = xs[(size_t)src * 3 * B + k];
    if (c_out) c_out[i] = cs[src];
    if (v_out) v_out[i] = vs[src];
}

// ------------------------------------------------------------------------------------
// Lift (damped least squares on the block frame) and trajectory seeding.
// ------------------------------------------------------------------------------------
// IK error of the block frame T_B = T_E G^-1 at q (position, then orientation: kind 0
// the z axis against e_z, kind 1 half the sum of axis cross products against Rz(yaw)),
// with the joint origins and axes o_{j-1}, z_{j-1} and the block origin for the Jacobian.
// P: the problem by reference (KProb) or through the constant address space (cKProb).
template <class KP>
__device__ __forceinline__ void ik_eval(const KP &P, int kind, float tx, float ty, float tz, float cy, float sy,
                                        const float (&q)[NJ], float (&ax)[NJ][6], float &t0, float &t1, float &t2,
                                        float (&e)[6])
{
    Frame F;
    frame_identity(F);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        ax[j][0] = F.p0; ax[j][1] = F.p1; ax[j][2] = F.p2;
        ax[j][3] = F.z0; ax[j][4] = F.z1; ax[j][5] = F.z2;
        dh_step(F, P.a[j], P.d[j], P.ca[j], P.sa[j], q[j]);
    }
    const float pe0 = F.p0 + P.tool_d * F.z0, pe1 = F.p1 + P.tool_d * F.z1, pe2 = F.p2 + P.tool_d * F.z2;
    const auto &Gr = P.Gi_R;
    float RB[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        RB[0][c] = Gr[c] * F.x0 + Gr[3 + c] * F.y0 + Gr[6 + c] * F.z0;
        RB[1][c] = Gr[c] * F.x1 + Gr[3 + c] * F.y1 + Gr[6 + c] * F.z1;
        RB[2][c] = Gr[c] * F.x2 + Gr[3 + c] * F.y2 + Gr[6 + c] * F.z2;
    }
    t0 = pe0 + P.Gi_t[0] * F.x0 + P.Gi_t[1] * F.y0 + P.Gi_t[2] * F.z0;
    t1 = pe1 + P.Gi_t[0] * F.x1 + P.Gi_t[1] * F.y1 + P.Gi_t[2] * F.z1;
    t2 = pe2 + P.Gi_t[0] * F.x2 + P.Gi_t[1] * F.y2 + P.Gi_t[2] * F.z2;
    e[0] = tx - t0;
    e[1] = ty - t1;
    e[2] = tz - t2;
    if (kind == 0) {
        // (R_B e_z) x e_z
        e[3] = RB[1][2];
        e[4] = -RB[0][2];
        e[5] = 0.f;
    } else {
        // 1/2 sum_c (R_B e_c) x (Rz(yaw) e_c)
        const float R0[3] = {cy, sy, 0.f}, R1[3] = {-sy, cy, 0.f};
        float w0 = 0.f, w1 = 0.f, w2 = 0.f;
        w0 += RB[1][0] * R0[2] - RB[2][0] * R0[1];
        w1 += RB[2][0] * R0[0] - RB[0][0] * R0[2];
        w2 += RB[0][0] * R0[1] - RB[1][0] * R0[0];
        w0 += RB[1][1] * R1[2] - RB[2][1] * R1[1];
        w1 += RB[2][1] * R1[0] - RB[0][1] * R1[2];
        w2 += RB[0][1] * R1[1] - RB[1][1] * R1[0];
        w0 += RB[1][2];   // (R_B e_z) x e_z
        w1 += -RB[0][2];
        e[3] = 0.5f * w0;
        e[4] = 0.5f * w1;
        e[5] = 0.5f * w2;
    }
}

template <class KP>
__device__ __forceinline__ float ik_error(const KP &P, int kind, float tx, float ty, float tz, float tyaw,
                                          const float (&q)[NJ])
{
    float sy, cy;
    sincosf(tyaw, &sy, &cy);
    float ax[NJ][6], t0, t1, t2, e[6];
    ik_eval(P, kind, tx, ty, tz, cy, sy, q, ax, t0, t1, t2, e);
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < 6; ++r) s += e[r] * e[r];
    return sqrtf(s);
}

// Not inlined: the single-iteration entry point and the multi-start lift then run the
// same instructions, so their iterates are bit-identical (inlined copies may contract
// multiply-adds differently once `kind` is a constant).  The problem comes as its device
// copy in the constant address space: a reference to the kernel's by-value argument
// would make every lane copy the whole struct to scratch memory.
typedef __attribute__((address_space(4))) const KProb cKProb;
__device__ __noinline__ void ik_run(const cKProb *Pc, int kind, float tx, float ty, float tz, float tyaw,
                                    float (&q)[NJ], int iters)
{
    const cKProb &P = *Pc;
    float sy, cy;
    sincosf(tyaw, &sy, &cy);
    const float lam2 = P.ik_lambda * P.ik_lambda;
    for (int it = 0; it < iters; ++it) {
        float ax[NJ][6], t0, t1, t2, e[6];
        ik_eval(P, kind, tx, ty, tz, cy, sy, q, ax, t0, t1, t2, e);
        // A = J J^T + lambda^2 I, J column j = (z x (t_B - o), z)
        float A[6][6];
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = 0; c < 6; ++c) A[r][c] = (r == c) ? lam2 : 0.f;
        float J[NJ][6];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const float r0 = t0 - ax[j][0], r1 = t1 - ax[j][1], r2 = t2 - ax[j][2];
            const float z0 = ax[j][3], z1 = ax[j][4], z2 = ax[j][5];
            J[j][0] = z1 * r2 - z2 * r1;
            J[j][1] = z2 * r0 - z0 * r2;
            J[j][2] = z0 * r1 - z1 * r0;
            J[j][3] = z0;
            J[j][4] = z1;
            J[j][5] = z2;
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int c = 0; c <= r; ++c) A[r][c] += J[j][r] * J[j][c];
        }
        // Cholesky A = L L^T (lower), then L L^T y = e
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            float s = A[c][c];
#pragma unroll
            for (int k = 0; k < c; ++k) s -= A[c][k] * A[c][k];
            const float d = sqrtf(fmaxf(s, 1e-30f));
            A[c][c] = d;
            const float inv = 1.f / d;
#pragma unroll
            for (int r = c + 1; r < 6; ++r) {
                float t = A[r][c];
#pragma unroll
                for (int k = 0; k < c; ++k) t -= A[r][k] * A[c][k];
                A[r][c] = t * inv;
            }
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            float t = e[r];
#pragma unroll
            for (int k = 0; k < r; ++k) t -= A[r][k] * e[k];
            e[r] = t / A[r][r];
        }
#pragma unroll
        for (int r = 5; r >= 0; --r) {
            float t = e[r];
#pragma unroll
            for (int k = r + 1; k < 6; ++k) t -= A[k][r] * e[k];
            e[r] = t / A[r][r];
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            float dq = 0.f;
#pragma unroll
            for (int r = 0; r < 6; ++r) dq += J[j][r] * e[r];
            q[j] = fminf(fmaxf(q[j] + dq, P.lo[j]), P.hi[j]);
        }
    }
}

__global__ void k_ik_iterate(KProb P, int kind, int n, const float *target, float *qio, int iters)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n) return;
    float q[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] = qio[(size_t)gid * NJ + j];
    const float *t = target + (size_t)gid * 4;
    ik_run((const cKProb *)P.self, kind, t[0], t[1], t[2], t[3], q, iters);
#pragma unroll
    for (int j = 0; j < NJ; ++j) qio[(size_t)gid * NJ + j] = q[j];
}

// How deep the arm stands in the clutter at q, for block b in situation kind (0 grasp,
// 1 place, 2 transit interior, 3 transfer interior): the sum over robot spheres of
// max(0, r - sdf) against every box and every block visible there -- blocks below b at
// their placements pose[bb], blocks above b at their initial poses, block b itself at its
// placement after the place and at its initial pose inside its transit.  Dense: it runs
// once per IK start or seed candidate.  Padded spheres (r = -1e30) contribute nothing.
__device__ __forceinline__ float arm_clutter(const KProb &P, const float (&q)[NJ], const float *pose, int b, int kind)
{
    Frame F;
    frame_identity(F);
    float pen = 0.f;
    const float half = P.half;
#pragma unroll
    for (int J = 0; J < NJ; ++J) {
        dh_step(F, P.a[J], P.d[J], P.ca[J], P.sa[J], q[J]);
        // obstacles: those that meet no lane's bounds of the link's spheres (1e-4 m margin)
        // contribute exactly zero and are skipped by the whole wave
        float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
        for (int s = P.link_start[J]; s < P.link_start[J + 1]; ++s) {
            const float4 sp = ldc(P.sph, s);
            const float cx = F.p0 + sp.x * F.x0 + sp.y * F.y0 + sp.z * F.z0;
            const float cy = F.p1 + sp.x * F.x1 + sp.y * F.y1 + sp.z * F.z1;
            const float cz = F.p2 + sp.x * F.x2 + sp.y * F.y2 + sp.z * F.z2;
            lo0 = fminf(lo0, cx - sp.w);
            lo1 = fminf(lo1, cy - sp.w);
            lo2 = fminf(lo2, cz - sp.w);
            hi0 = fmaxf(hi0, cx + sp.w);
            hi1 = fmaxf(hi1, cy + sp.w);
            hi2 = fmaxf(hi2, cz + sp.w);
        }
        for (int o = 0; o < P.O; ++o) {
            const float4 bl = ldc(P.box, 4 * o + 2), bh = ldc(P.box, 4 * o + 3);
            if (!__any((bl.x <= hi0 + 1e-4f) & (bh.x >= lo0 - 1e-4f) & (bl.y <= hi1 + 1e-4f) & (bh.y >= lo1 - 1e-4f) &
                       (bl.z <= hi2 + 1e-4f) & (bh.z >= lo2 - 1e-4f)))
                continue;
            const float4 bc = ldc(P.box, 4 * o), be = ldc(P.box, 4 * o + 1);
            for (int s = P.link_start[J]; s < P.link_start[J + 1]; ++s) {
                const float4 sp = ldc(P.sph, s);
                const float cx = F.p0 + sp.x * F.x0 + sp.y * F.y0 + sp.z * F.z0;
                const float cy = F.p1 + sp.x * F.x1 + sp.y * F.y1 + sp.z * F.z1;
                const float cz = F.p2 + sp.x * F.x2 + sp.y * F.y2 + sp.z * F.z2;
                const float ux = fabsf(cx - bc.x) - be.x, uy = fabsf(cy - bc.y) - be.y, uz = fabsf(cz - bc.z) - be.z;
                const float qx = fmaxf(ux, 0.f), qy = fmaxf(uy, 0.f), qz = fmaxf(uz, 0.f);
                const float sdf = __builtin_amdgcn_sqrtf(qx * qx + qy * qy + qz * qz) + fminf(fmaxf(fmaxf(ux, uy), uz), 0.f);
                pen += fmaxf(sp.w - sdf, 0.f);
            }
        }
        for (int s = P.link_start[J]; s < P.link_start[J + 1]; ++s) {
            const float4 sp = ldc(P.sph, s);
            const float cx = F.p0 + sp.x * F.x0 + sp.y * F.y0 + sp.z * F.z0;
            const float cy = F.p1 + sp.x * F.x1 + sp.y * F.y1 + sp.z * F.z1;
            const float cz = F.p2 + sp.x * F.x2 + sp.y * F.y2 + sp.z * F.z2;
            for (int bb = 0; bb < (P.mode == SPASM_MODE_P2P ? 0 : P.B); ++bb) {  // p2p: no blocks
                float tx, ty, tz, yaw;
                if (bb < b || (bb == b && kind == 1)) {
                    tx = pose[4 * bb];
                    ty = pose[4 * bb + 1];
                    tz = pose[4 * bb + 2];
                    yaw = pose[4 * bb + 3];
                } else if (bb > b || (bb == b && kind == 2)) {
                    const float4 I = ldc(P.blk_init, 2 * bb);
                    tx = I.x;
                    ty = I.y;
                    tz = I.z;
                    yaw = I.w;
                } else {
                    continue;
                }
                float sn, cs;
                sincosf(yaw, &sn, &cs);
                const float dx = cx - tx, dy = cy - ty, dz = cz - tz;
                const float lx = cs * dx + sn * dy, ly = cs * dy - sn * dx;
                const float ux = fabsf(lx) - half, uy = fabsf(ly) - half, uz = fabsf(dz) - half;
                const float qx = fmaxf(ux, 0.f), qy = fmaxf(uy, 0.f), qz = fmaxf(uz, 0.f);
                const float sdf = __builtin_amdgcn_sqrtf(qx * qx + qy * qy + qz * qz) + fminf(fmaxf(fmaxf(ux, uy), uz), 0.f);
                pen += fmaxf(sp.w - sdf, 0.f);
            }
        }
    }
    return pen;
}

// Multi-start lift: eight lanes per (particle, block), lane r runs start r < restarts
// (start 0 from q_home + noise, resp. from the chosen grasp; the others uniform over the
// limits).  Among the starts whose error is below 1e-4 the group keeps the one standing
// least deep in the obstacles (first on ties); when none converged, the smallest error
// (first on ties).  The choice is broadcast to the group.
__device__ __forceinline__ int ik_pick(float err, float pen, int r, int restarts)
{
    const int lane = threadIdx.x & 63, g0 = lane & ~7;
    const bool ok = r < restarts && err < 1e-4f;
    const unsigned long long acc = (__ballot(ok) >> g0) & 0xFFull;
    if (acc) {
        const float sc = ok ? pen : INFINITY;
        const float m = group8_reduce(sc, OpMin());
        return g0 + __builtin_ctzll((__ballot(ok && sc == m) >> g0) & 0xFFull);
    }
    const float e = r < restarts ? err : INFINITY;
    const float m = group8_reduce(e, OpMin());
    const unsigned long long at = (__ballot(e == m) >> g0) & 0xFFull;
    return g0 + __builtin_ctzll(at);
}

__global__ __launch_bounds__(256) void k_ik_lift(KProb P, int nP, const float *pose, uint64_t seed, int iters,
                                                 float *qg, float *qp)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = gid >> 3, r = gid & 7;
    if (grp >= nP * P.B) return;  // whole 8-lane groups only
    const int B = P.B, p = grp / B, b = grp % B, R = P.ik_restarts;
    float u[8], q[NJ];
    uniforms4(seed, (uint64_t)p, (uint64_t)(2 * b), (uint64_t)r, 2u, u);
    uniforms4(seed, (uint64_t)p, (uint64_t)(2 * b + 1), (uint64_t)r, 2u, u + 4);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        q[j] = r == 0 ? fminf(fmaxf(P.q_home[j] + P.ik_noise * (2.f * u[j] - 1.f), P.lo[j]), P.hi[j])
                      : P.lo[j] + (P.hi[j] - P.lo[j]) * u[j];
    const float4 I = ldc(P.blk_init, 2 * b);
    float err = INFINITY, pen = 0.f;
    if (r < R) {
        ik_run((const cKProb *)P.self, 0, I.x, I.y, I.z, 0.f, q, iters);
        err = ik_error(P, 0, I.x, I.y, I.z, 0.f, q);
        if (err < 1e-4f) pen = arm_clutter(P, q, pose + (size_t)p * B * 4, b, 0);
    }
    int src = ik_pick(err, pen, r, R);
    float qc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) qc[j] = __shfl(q[j], src, 64);
    if (r == 0) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) qg[(size_t)grp * NJ + j] = qc[j];
    }
    uniforms4(seed, (uint64_t)p, (uint64_t)(2 * B + 2 * b), (uint64_t)r, 2u, u);
    uniforms4(seed, (uint64_t)p, (uint64_t)(2 * B + 2 * b + 1), (uint64_t)r, 2u, u + 4);
#pragma unroll
    for (int j = 0; j < NJ; ++j) q[j] = r == 0 ? qc[j] : P.lo[j] + (P.hi[j] - P.lo[j]) * u[j];
    const float *t = pose + (size_t)grp * 4;
    err = INFINITY;
    pen = 0.f;
    if (r < R) {
        ik_run((const cKProb *)P.self, 1, t[0], t[1], t[2], t[3], q, iters);
        err = ik_error(P, 1, t[0], t[1], t[2], t[3], q);
        if (err < 1e-4f) pen = arm_clutter(P, q, pose + (size_t)p * B * 4, b, 1);
    }
    src = ik_pick(err, pen, r, R);
#pragma unroll
    for (int j = 0; j < NJ; ++j) qc[j] = __shfl(q[j], src, 64);
    if (r == 0) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) qp[(size_t)grp * NJ + j] = qc[j];
    }
}

// Segment ends (start, goal) of segment s of particle p.
__device__ __forceinline__ void segment_ends(const KProb &P, const float *qg, const float *qp, int p, int s,
                                             float (&qa)[NJ], float (&qb)[NJ])
{
    const int B = P.B, b = s >> 1;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (P.mode == SPASM_MODE_P2P) {  // the one motion: start to goal
            qa[j] = fminf(fmaxf(P.q_home[j], P.lo[j]), P.hi[j]);
            qb[j] = fminf(fmaxf(P.p2p_goal[j], P.lo[j]), P.hi[j]);
        } else if (s & 1) {
            qa[j] = qg[((size_t)p * B + b) * NJ + j];
            qb[j] = qp[((size_t)p * B + b) * NJ + j];
        } else {
            qa[j] = b == 0 ? fminf(fmaxf(P.q_home[j], P.lo[j]), P.hi[j]) : qp[((size_t)p * B + b - 1) * NJ + j];
            qb[j] = qg[((size_t)p * B + b) * NJ + j];
        }
    }
}

// Intermediate waypoint of each segment: 32 lanes per (particle, segment), four per
// candidate c < 8.  Candidate c < mid_candidates draws the ends' midpoint + noise
// (counter (p, 2s + chunk, c, 3)) and is scored by arm-obstacle penetration at the draw
// and at the two points halfway to the ends, one point per lane (the fourth lane adds
// zero, so the sum is (draw + first half point) + second half point in every case); the
// lowest score (first candidate on ties) is written to waypoint (W-1)/2.
__global__ __launch_bounds__(256) void k_seed_mid(KProb P, int nP, int W, const float *qg, const float *qp,
                                                  const float *pose, uint64_t seed, float *q)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = gid >> 5, c = (gid >> 2) & 7, pt = gid & 3, NS = n_segments(P), C = P.mid_candidates;
    if (grp >= nP * NS) return;  // whole 32-lane groups only
    const int p = grp / NS, s = grp % NS;
    float qa[NJ], qb[NJ], qc[NJ], qe[NJ], u[8];
    segment_ends(P, qg, qp, p, s, qa, qb);
    uniforms4(seed, (uint64_t)p, (uint64_t)(2 * s), (uint64_t)c, 3u, u);
    uniforms4(seed, (uint64_t)p, (uint64_t)(2 * s + 1), (uint64_t)c, 3u, u + 4);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        qc[j] = fminf(fmaxf(0.5f * (qa[j] + qb[j]) + P.mid_noise * (2.f * u[j] - 1.f), P.lo[j]), P.hi[j]);
        qe[j] = pt == 0 ? qc[j] : pt == 1 ? 0.5f * (qa[j] + qc[j]) : 0.5f * (qc[j] + qb[j]);
    }
    float part = 0.f;
    if (c >= C) {
        part = INFINITY;
    } else if (C > 1 && pt < 3) {
        const float *pp = pose ? pose + (size_t)p * P.B * 4 : nullptr;  // p2p: no blocks, unused
        const int kind = 2 + (s & 1);  // transit or transfer interior
        part = arm_clutter(P, qe, pp, s >> 1, kind);
    }
    const float sc = part + __shfl_xor(part, 1, 64);
    const float tot = sc + __shfl_xor(sc, 2, 64);
    float best = tot;
    best = fminf(best, __shfl_xor(best, 4, 64));
    best = fminf(best, __shfl_xor(best, 8, 64));
    best = fminf(best, __shfl_xor(best, 16, 64));
    const int lane = threadIdx.x & 63, g0 = lane & ~31;
    const unsigned long long hit = __ballot(pt == 0 && c < C && tot == best);
    const int src = g0 + __builtin_ctzll((hit >> g0) & 0xFFFFFFFFull);
    float qm[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) qm[j] = __shfl(qc[j], src, 64);
    if (c == 0 && pt == 0) {
        float *o = q + (((size_t)p * NS + s) * W + (W - 1) / 2) * NJ;
#pragma unroll
        for (int j = 0; j < NJ; ++j) o[j] = qm[j];
    }
}

// Straight lines start -> intermediate (read from waypoint (W-1)/2, left as it is) -> goal.
__global__ void k_traj_init(KProb P, int nP, int W, const float *qg, const float *qp, uint64_t seed, float *q)
{
    const int B = P.B, NS = n_segments(P);
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nP * NS * W) return;
    const int w = gid % W, s = (gid / W) % NS, p = gid / (W * NS);
    const int m = (W - 1) / 2;
    if (w == m) return;  // the chosen intermediate waypoint
    (void)B;
    (void)seed;
    float qa[NJ], qb[NJ];
    segment_ends(P, qg, qp, p, s, qa, qb);
    const float *mid = q + (((size_t)p * NS + s) * W + m) * NJ;
    float *o = q + (size_t)gid * NJ;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const float qm = mid[j];
        float v;
        if (w == 0)
            v = qa[j];
        else if (w == W - 1)
            v = qb[j];
        else if (w < m)
            v = qa[j] + ((float)w / (float)m) * (qm - qa[j]);
        else
            v = qm + ((float)(w - m) / (float)(W - 1 - m)) * (qb[j] - qm);
        o[j] = v;
    }
}

// ------------------------------------------------------------------------------------
// Solve glue
// ------------------------------------------------------------------------------------
// Commit a stage-1 round: if no earlier round committed and this one has satisfying
// particles (or is the last), its particles in satisfying-first order become the stage-2
// placements (z at the slot height).  info: [0] stage-1 satisfying count, [1] rounds.
__global__ __launch_bounds__(1024) void k_commit_stage1(KProb P, int M, int round, int last, const float *xs,
                                                        const float *cs, const float *vs, const int32_t *order,
                                                        const int32_t *nsat, float *pose, float *cost_out,
                                                        float *viol_out, int *done, int32_t *info)
{
    __shared__ int s_go;
    if (threadIdx.x == 0) s_go = (*done == 0) && (*nsat > 0 || last);
    __syncthreads();
    if (!s_go) return;
    const int B = P.B;
    for (int e = threadIdx.x; e < M * B; e += blockDim.x) {
        const int m = e / B, b = e % B;
        const float *x = xs + ((size_t)order[m] * B + b) * 3;
        float *o = pose + ((size_t)m * B + b) * 4;
        o[0] = x[0];
        o[1] = x[1];
        o[2] = zstar(P, b);
        o[3] = x[2];
    }
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        if (cost_out) cost_out[m] = cs[order[m]];
        if (viol_out) viol_out[m] = vs[order[m]];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *done = 1;
        info[0] = *nsat;
        info[1] = round + 1;
    }
}

__global__ void k_fixed_poses(KProb P, int M, float *pose, int32_t *info)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) {
        info[0] = -1;
        info[1] = 0;
    }
    if (gid >= M * P.B) return;
    const int b = gid % P.B;
    const float4 g = ldc(P.goal, 2 * b);
    float *o = pose + (size_t)gid * 4;
    o[0] = g.x;
    o[1] = g.y;
    o[2] = g.z;
    o[3] = g.w;
}

// Best particle (first in satisfying-first order): copy it out, path length.
// info: [2] n_sat, [3] best; finfo: [0] viol, [1] cost, [2] length
__global__ __launch_bounds__(1024) void k_finalize(KProb P, int M, int W, const float *q, const float *pose,
                                                   const float *cost, const float *viol, const int32_t *order,
                                                   const int32_t *nsat, float *best_q, float *best_pose, int32_t *info,
                                                   float *finfo)
{
    __shared__ float s_len[16];
    const int B = P.B, NS = n_segments(P), tid = threadIdx.x;
    const int best = order[0];
    const float *qb = q + (size_t)best * NS * W * NJ;
    for (int e = tid; e < NS * W * NJ; e += blockDim.x) best_q[e] = qb[e];
    if (tid < 4 * B && best_pose) best_pose[tid] = pose[(size_t)best * 4 * B + tid];
    float len = 0.f;
    for (int e = tid; e < NS * W; e += blockDim.x) {
        const int w = e % W;
        if (w == W - 1) continue;
        float ss = 0.f;
        for (int j = 0; j < NJ; ++j) {
            const float d = qb[(e + 1) * NJ + j] - qb[e * NJ + j];
            ss += d * d;
        }
        len += sqrtf(ss);
    }
    len = wave_sum(len);
    if ((tid & 63) == 0) s_len[tid >> 6] = len;
    __syncthreads();
    if (tid == 0) {
        float L = 0.f;
        for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) L += s_len[wv];
        info[2] = *nsat;
        info[3] = best;
        finfo[0] = viol[best];
        finfo[1] = cost[best];
        finfo[2] = L;
    }
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
static int lcm_int(int a, int b)
{
    int x = a, y = b;
    while (y) {
        const int t = x % y;
        x = y;
        y = t;
    }
    return a / x * b;
}

hipError_t launch_sample(const KProb &P, int N, uint64_t seed, int round, float *x, const int *skip, hipStream_t st)
{
    const int n = N * P.B;
    hipLaunchKernelGGL(k_sample, dim3((n + 255) / 256), dim3(256), 0, st, P, N, seed, round, x, skip);
    return hipGetLastError();
}

hipError_t launch_place(const KProb &P, int n, const float *x_in, const int32_t *idx, float *x_out, int k_begin,
                        int k_end, int eval_phase, float *cost, float *viol, float *gx, const int *skip, hipStream_t st)
{
    const int L = 1 << P.lpb_log2, per = P.B * L, threads = lcm_int(per, 64), ppw = threads / per;
    // state and reduction per block; packing adds the cells (float4 each) and the pair
    // gradients left for other pieces (3 floats per piece and offset t = 1..B/2)
    const bool pack = P.mode == SPASM_MODE_PACK;
    const size_t shm = (size_t)ppw * P.B * (10 + (pack ? 4 * L + 3 * (P.B / 2) : 0)) * sizeof(float);
    hipLaunchKernelGGL(k_place, dim3((n + ppw - 1) / ppw), dim3(threads), shm, st, P, n, x_in, idx, x_out, k_begin,
                       k_end, eval_phase, cost, viol, gx, skip);
    return hipGetLastError();
}

int traj_threads(int B, int W) { return ((2 * B * W + 63) / 64) * 64; }

// The optimisation launch's register bound for particles of `threads` lanes (see k_traj).
static bool opt_bound_768(int threads)
{
    const int w = threads / 64;
    return w <= 12 && 12 / w == 16 / w;
}

template <int CH>
static hipError_t launch_traj_ch(const KProb &P, int mode, const TrajArgs &a, hipStream_t st)
{
    const int threads = traj_threads(P.B, a.W);
    if (mode == 0)
        hipLaunchKernelGGL((k_traj<0, CH>), dim3(a.P), dim3(threads), 0, st, P, a);
    else if (mode == 1)
        hipLaunchKernelGGL((k_traj<1, CH>), dim3(a.P), dim3(threads), 0, st, P, a);
    else if (opt_bound_768(threads))
        hipLaunchKernelGGL((k_traj<2, CH, 768>), dim3(a.P), dim3(threads), (size_t)2 * NJ * threads * sizeof(float),
                           st, P, a);
    else
        hipLaunchKernelGGL((k_traj<2, CH>), dim3(a.P), dim3(threads), (size_t)2 * NJ * threads * sizeof(float), st,
                           P, a);
    return hipGetLastError();
}

hipError_t launch_traj(const KProb &P, int mode, const TrajArgs &a, hipStream_t st)
{
    // the sphere table is padded so that every link holds a multiple of P.chunk spheres
    switch (P.chunk) {
    case 4: return launch_traj_ch<4>(P, mode, a, st);
    case 6: return launch_traj_ch<6>(P, mode, a, st);
    case 7: return launch_traj_ch<7>(P, mode, a, st);
    case 8: return launch_traj_ch<8>(P, mode, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int CH>
static void launch_serve_ch(int threads, int nwg, const ServeSolve *d_solves, int nsolve, hipStream_t st)
{
    // the same register bound as the plain optimisation launch of this shape, so that a
    // served particle runs the same instructions
    const size_t shm = (size_t)2 * NJ * threads * sizeof(float);
    if (opt_bound_768(threads))
        hipLaunchKernelGGL((k_serve<CH, 768>), dim3(nwg), dim3(threads), shm, st, d_solves, nsolve);
    else
        hipLaunchKernelGGL((k_serve<CH, 1024>), dim3(nwg), dim3(threads), shm, st, d_solves, nsolve);
}

hipError_t launch_serve(int chunk, int threads, int nwg, const ServeSolve *d_solves, int nsolve, hipStream_t st)
{
    switch (chunk) {
    case 4: launch_serve_ch<4>(threads, nwg, d_solves, nsolve, st); break;
    case 6: launch_serve_ch<6>(threads, nwg, d_solves, nsolve, st); break;
    case 7: launch_serve_ch<7>(threads, nwg, d_solves, nsolve, st); break;
    case 8: launch_serve_ch<8>(threads, nwg, d_solves, nsolve, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t set_smem_limits(size_t sort_bytes, size_t traj_bytes)
{
    hipError_t e = hipFuncSetAttribute((const void *)k_rank_sort, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(sort_bytes + 16 * 64 * sizeof(uint32_t)));
    if (e != hipSuccess) return e;
#define SPASM_TRAJ_ATTR(CH)                                                                                      \
    e = hipFuncSetAttribute((const void *)k_traj<2, CH>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)traj_bytes); \
    if (e != hipSuccess) return e;                                                                           \
    e = hipFuncSetAttribute((const void *)k_traj<2, CH, 768>, hipFuncAttributeMaxDynamicSharedMemorySize,     \
                            (int)traj_bytes);                                                                \
    if (e != hipSuccess) return e;                                                                           \
    e = hipFuncSetAttribute((const void *)k_serve<CH, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize,      \
                            (int)traj_bytes);                                                                \
    if (e != hipSuccess) return e;                                                                           \
    e = hipFuncSetAttribute((const void *)k_serve<CH, 768>, hipFuncAttributeMaxDynamicSharedMemorySize,       \
                            (int)traj_bytes);                                                                \
    if (e != hipSuccess) return e;
    SPASM_TRAJ_ATTR(4)
    SPASM_TRAJ_ATTR(6)
    SPASM_TRAJ_ATTR(7)
    SPASM_TRAJ_ATTR(8)
#undef SPASM_TRAJ_ATTR
    return hipSuccess;
}

// Rank selection over n <= 16384 keys: KB keys per workgroup (16, 32 or 64, so that up
// to 256 workgroups share the work); the first nout sorted indices are written.
static hipError_t launch_sort(int kind, int n, const float *cost, const float *viol, float eps,
                              const unsigned long long *in_keys, int nout, int32_t *out_idx, int32_t *out_count,
                              const int *skip, hipStream_t st)
{
    if (n < 1 || n > MAX_SORT || nout > n) return hipErrorInvalidValue;
    const int kb_log2 = n <= 4096 ? 4 : n <= 8192 ? 5 : 6;
    const int grid = (n + (1 << kb_log2) - 1) >> kb_log2;
    const size_t shm = (size_t)n * sizeof(unsigned long long) + 16 * 64 * sizeof(uint32_t);
    hipLaunchKernelGGL(k_rank_sort, dim3(grid), dim3(1024), shm, st, kind, n, kb_log2, cost, viol, eps, in_keys, nout,
                       out_idx, out_count, skip);
    return hipGetLastError();
}

hipError_t launch_sort_keys(int kind, int n, const float *cost, const float *viol, float eps, int M,
                            int32_t *out_idx, int32_t *out_count, const int *skip, hipStream_t st)
{
    return launch_sort(kind, n, cost, viol, eps, nullptr, kind == 0 ? M : n, out_idx, out_count, skip, st);
}

static size_t align_up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of the radix select: state (4 words) in the first 256 bytes, the 2048-bin
// histogram, the per-workgroup counts of keys below and equal to T, then M 64-bit keys.
size_t topm_workspace(int n, int M)
{
    if (n <= MAX_SORT) return 0;
    const size_t G = (size_t)(n + RS_KEYS - 1) / RS_KEYS;
    return 256 + 2048 * sizeof(uint32_t) + align_up256(2 * G * sizeof(uint32_t)) + (size_t)M * sizeof(unsigned long long);
}

hipError_t launch_topm(int n, const float *cost, int M, int32_t *out_idx, void *ws, hipStream_t st)
{
    if (n <= MAX_SORT) return launch_sort_keys(0, n, cost, nullptr, 0.f, M, out_idx, nullptr, nullptr, st);
    const int G = (n + RS_KEYS - 1) / RS_KEYS;
    char *w = (char *)ws;
    uint32_t *state = (uint32_t *)w;
    uint32_t *hist = (uint32_t *)(w + 256);
    uint32_t *wg_lt = (uint32_t *)(w + 256 + 2048 * sizeof(uint32_t)), *wg_eq = wg_lt + G;
    unsigned long long *surv =
        (unsigned long long *)(w + 256 + 2048 * sizeof(uint32_t) + align_up256(2 * (size_t)G * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_rs_init, dim3(1), dim3(1024), 0, st, M, state, hist);
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(k_rs_hist, dim3(G), dim3(1024), 0, st, n, cost, pass, (const uint32_t *)state, hist);
        hipLaunchKernelGGL(k_rs_pick, dim3(1), dim3(1024), 0, st, pass, state, hist);
    }
    hipLaunchKernelGGL(k_rs_count, dim3(G), dim3(1024), 0, st, n, cost, (const uint32_t *)state, wg_lt, wg_eq);
    hipLaunchKernelGGL(k_rs_collect, dim3(G), dim3(1024), 0, st, n, cost, (const uint32_t *)state,
                       (const uint32_t *)wg_lt, (const uint32_t *)wg_eq, M, surv);
    return launch_sort(2, M, nullptr, nullptr, 0.f, surv, M, out_idx, nullptr, nullptr, st);
}

hipError_t launch_gather_place(int B, int M, const float *xs, const float *cs, const float *vs, const int32_t *ord,
                               float *x_out, float *c_out, float *v_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_place, dim3((M + 255) / 256), dim3(256), 0, st, B, M, xs, cs, vs, ord, x_out, c_out,
                       v_out);
    return hipGetLastError();
}

hipError_t launch_ik_iterate(const KProb &P, int kind, int n, const float *target, float *q, int iters, hipStream_t st)
{
    hipLaunchKernelGGL(k_ik_iterate, dim3((n + 127) / 128), dim3(128), 0, st, P, kind, n, target, q, iters);
    return hipGetLastError();
}

hipError_t launch_ik_lift(const KProb &P, int nP, const float *pose, uint64_t seed, int iters, float *qg, float *qp,
                          hipStream_t st)
{
    const long n = (long)nP * P.B * 8;
    hipLaunchKernelGGL(k_ik_lift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, nP, pose, seed, iters, qg, qp);
    return hipGetLastError();
}

hipError_t launch_traj_init(const KProb &P, int nP, int W, const float *qg, const float *qp, const float *pose,
                            uint64_t seed, float *q, hipStream_t st)
{
    const long g = (long)nP * 2 * P.B * 32;  // 32 lanes per (particle, segment); p2p groups past NS exit
    hipLaunchKernelGGL(k_seed_mid, dim3((unsigned)((g + 255) / 256)), dim3(256), 0, st, P, nP, W, qg, qp, pose, seed,
                       q);
    const int n = nP * 2 * P.B * W;
    hipLaunchKernelGGL(k_traj_init, dim3((n + 255) / 256), dim3(256), 0, st, P, nP, W, qg, qp, seed, q);
    return hipGetLastError();
}

hipError_t launch_commit_stage1(const KProb &P, int M, int round, int last_round, const float *xs,
                                const float *cs, const float *vs, const int32_t *order, const int32_t *nsat,
                                float *pose, float *cost_out, float *viol_out, int *done, int32_t *info,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_commit_stage1, dim3(1), dim3(1024), 0, st, P, M, round, last_round, xs, cs, vs, order, nsat,
                       pose, cost_out, viol_out, done, info);
    return hipGetLastError();
}

__global__ void k_check_stop(const int32_t *nsat, int32_t *done, int32_t *stop_iter, int iters)
{
    if (threadIdx.x == 0 && *done == 0 && *nsat > 0) {
        *done = 1;
        *stop_iter = iters;
    }
}

hipError_t launch_check_stop(const int32_t *nsat, int32_t *done, int32_t *stop_iter, int iters, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_stop, dim3(1), dim3(64), 0, st, nsat, done, stop_iter, iters);
    return hipGetLastError();
}

hipError_t launch_fixed_poses(const KProb &P, int M, float *pose, int32_t *info, hipStream_t st)
{
    const int n = M * P.B;
    hipLaunchKernelGGL(k_fixed_poses, dim3((n + 255) / 256), dim3(256), 0, st, P, M, pose, info);
    return hipGetLastError();
}

hipError_t launch_finalize(const KProb &P, int M, int W, const float *q, const float *pose, const float *cost,
                           const float *viol, const int32_t *order, const int32_t *nsat, float *best_q,
                           float *best_pose, int32_t *info, float *finfo, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, P, M, W, q, pose, cost, viol, order, nsat, best_q,
                       best_pose, info, finfo);
    return hipGetLastError();
}

}  // namespace spasm
