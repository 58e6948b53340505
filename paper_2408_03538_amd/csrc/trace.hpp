// Packet traversal of the LBVH shared by the forward, bounce and adjoint
// kernels, and the per-ray Gaussian test.
//
// A wavefront traces 64 rays at once: 64 / G directions for each of G
// Morton-adjacent source splats (the "group" split of transfer.hip).  The
// wave walks the tree together: a child is entered if the ray of any live
// lane crosses its box, so node and Gaussian records are read at
// wave-uniform addresses (scalar loads, one per wave instead of one per
// lane), the control flow never diverges, and the traversal stack is one
// VGPR -- entry k lives in lane k (a lane-select write, a readlane read).
// Every lane still applies the exact per-ray hit test of its own ray at each
// visited Gaussian, so the result does not depend on which other rays share
// the wave.
#pragma once

#include "common.hpp"

namespace prtgs {

struct RayDir {
    float wx, wy, wz;     // direction
    float ix, iy, iz;     // component-wise reciprocal, zeros nudged to tiny values
};

__device__ inline RayDir make_dir(float wx, float wy, float wz)
{
    RayDir d;
    d.wx = wx;
    d.wy = wy;
    d.wz = wz;
    const float tiny = 1e-20f;
    d.ix = 1.0f / (fabsf(wx) > tiny ? wx : copysignf(tiny, wx));
    d.iy = 1.0f / (fabsf(wy) > tiny ? wy : copysignf(tiny, wy));
    d.iz = 1.0f / (fabsf(wz) > tiny ? wz : copysignf(tiny, wz));
    return d;
}

// Octant of a direction: bit k set iff component k of the reciprocal is >= 0.
__device__ inline int octant(const RayDir& d)
{
    return (d.ix >= 0.0f ? 1 : 0) | (d.iy >= 0.0f ? 2 : 0) | (d.iz >= 0.0f ? 4 : 0);
}

// Whether the ray o + t w crosses the box within [tlo, thi] (general form).
__device__ inline bool slab_hit(float lx, float ly, float lz, float hx, float hy, float hz, const RayDir& d,
                                float oix, float oiy, float oiz, float tlo, float thi)
{
    float x0 = fmaf(lx, d.ix, -oix), x1 = fmaf(hx, d.ix, -oix);
    float y0 = fmaf(ly, d.iy, -oiy), y1 = fmaf(hy, d.iy, -oiy);
    float z0 = fmaf(lz, d.iz, -oiz), z1 = fmaf(hz, d.iz, -oiz);
    float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), tlo));
    float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fminf(fmaxf(z0, z1), thi));
    return tn <= tf;
}

// The same when the wave's rays share one octant: the entry and exit planes
// (near / far corner) are chosen once per wave, on the scalar unit.
__device__ inline bool slab_hit_oct(float nx, float ny, float nz, float fx, float fy, float fz, const RayDir& d,
                                    float oix, float oiy, float oiz, float tlo, float thi)
{
    float tn = fmaxf(fmaxf(fmaf(nx, d.ix, -oix), fmaf(ny, d.iy, -oiy)), fmaxf(fmaf(nz, d.iz, -oiz), tlo));
    float tf = fminf(fminf(fmaf(fx, d.ix, -oix), fmaf(fy, d.iy, -oiy)), fminf(fmaf(fz, d.iz, -oiz), thi));
    return tn <= tf;
}

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per-ray work of a single-ray depth-first traversal of the same tree in
// the same order: child-box tests of the internal nodes the ray enters, and
// Gaussian tests of the leaves whose boxes it crosses.
struct RayCounts {
    uint32_t box_tests = 0;
    uint32_t prim_tests = 0;
    uint32_t wave_nodes = 0;    // internal nodes the wave visited (same in every lane)
    uint32_t wave_leaves = 0;   // Gaussian records the wave visited
};

// Walks the BVH for the wave's rays.  `live` is the lane's participation
// (may be cleared by `leaf`), [tlo, thi] the lane's ray interval (may be
// narrowed by `leaf`, through the references).  leaf(r, box_hit) is called,
// uniformly, for every leaf rank r whose box is crossed by a live lane;
// box_hit tells whether this lane's ray crosses it.  `order_dir` (uniform)
// orders the children (nearer first).  With kOct every ray of the wave lies
// in octant `oct`.  With kCount the lane's own single-ray work is tallied in
// `cnt` (the wave stack then also carries, per entry, whether this lane's
// ray entered that node).
//
// kStep orders each step's work; the walk and its results are the same, the
// kernels around it compile and run best with different orders (measured):
//   kLeavesFirst  the leaf children's Gaussian tests, then the choice of the
//                 next node, its load at the top of the next step (adjoint);
//   kChooseFirst  the choice, the leaves' tests, then the load (direct pass,
//                 8 waves per SIMD);
//   kLoadFirst    the choice and the load, then the leaves' tests, which the
//                 load then overlaps (the bounce walks, 4-5 waves per SIMD,
//                 which wait on the latency of the dependent node loads).
enum TraverseStep { kLeavesFirst, kChooseFirst, kLoadFirst };
template <bool kCount, bool kOct, int kStep, class LeafFn>
__device__ inline void packet_traverse(const Node* __restrict__ nodes, int n, const RayDir& d, float ox, float oy,
                                       float oz, bool& live, float& tlo, float& thi, unsigned* flags, LeafFn&& leaf,
                                       RayCounts* cnt, const float* order_dir, int oct)
{
    if (n == 1) {
        if (__ballot(live)) {
            if (kCount && live) cnt->prim_tests++;
            if (kCount) cnt->wave_leaves++;
            leaf(0, live);
        }
        return;
    }
    const float oix = ox * d.ix, oiy = oy * d.iy, oiz = oz * d.iz;
    const bool sx = oct & 1, sy = oct & 2, sz = oct & 4;
    const int my_lane = __lane_id();
    int stack = 0;           // entry k of the wave's stack lives in lane k
    uint64_t stack_in = 0;   // (kCount) whether this lane's ray entered entry k's node, bit per entry
    int sp = 0;
    bool inside = live;      // (kCount) this lane's ray entered the current node
    // A depth-first walk enters each of the n - 1 internal nodes at most once;
    // the cap (and the reference check) only guard against a malformed tree.
    int budget = n;
    int node = 0;   // the root
    Node nd;
    if constexpr (kStep != kLeavesFirst) nd = uniform_load(nodes, node);
    while (true) {
        if (--budget < 0) {
            raise_flag(flags, PRTGS_FLAG_BAD_TREE);
            break;
        }
        if constexpr (kStep == kLeavesFirst) nd = uniform_load(nodes, node);
        if (kCount) cnt->wave_nodes++;
        // both tests for every lane, no short-circuit: no divergent branch
        bool hl, hr;
        if (kOct) {
            hl = slab_hit_oct(sx ? nd.a.x : nd.a.w, sy ? nd.a.y : nd.b.x, sz ? nd.a.z : nd.b.y,
                              sx ? nd.a.w : nd.a.x, sy ? nd.b.x : nd.a.y, sz ? nd.b.y : nd.a.z, d, oix, oiy, oiz, tlo,
                              thi);
            hr = slab_hit_oct(sx ? nd.b.z : nd.c.y, sy ? nd.b.w : nd.c.z, sz ? nd.c.x : nd.c.w,
                              sx ? nd.c.y : nd.b.z, sy ? nd.c.z : nd.b.w, sz ? nd.c.w : nd.c.x, d, oix, oiy, oiz, tlo,
                              thi);
        } else {
            hl = slab_hit(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, d, oix, oiy, oiz, tlo, thi);
            hr = slab_hit(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, d, oix, oiy, oiz, tlo, thi);
        }
        hl = hl & live;
        hr = hr & live;
        if (kCount) {
            if (inside && live) cnt->box_tests += 2;
            hl = hl && inside;
            hr = hr && inside;
        }
        bool any_l = __ballot(hl) != 0ull;
        bool any_r = __ballot(hr) != 0ull;
        const int ref_l = nd.d.x, ref_r = nd.d.y;
        if (ref_l >= n - 1 || ~ref_l >= n || ref_r >= n - 1 || ~ref_r >= n) {
            raise_flag(flags, PRTGS_FLAG_BAD_TREE);
            break;
        }
        // The leaf children are visited in this step; the walk then goes on
        // with an internal child or the top of the stack.  (The two forms of
        // the leaf conditions compile differently; each order takes the one
        // that measured faster for its kernels.)
        bool leaf_l = false, leaf_r = false;
        if constexpr (kStep == kLeavesFirst) {
            if (any_l && ref_l < 0) {
                if (kCount && hl && live) cnt->prim_tests++;
                if (kCount) cnt->wave_leaves++;
                leaf(~ref_l, hl);
                any_l = false;
            }
            if (any_r && ref_r < 0) {
                if (kCount && hr && live) cnt->prim_tests++;
                if (kCount) cnt->wave_leaves++;
                leaf(~ref_r, hr);
                any_r = false;
            }
        } else {
            leaf_l = any_l && ref_l < 0;
            leaf_r = any_r && ref_r < 0;
            if (leaf_l) any_l = false;
            if (leaf_r) any_r = false;
        }
        int next = -1;
        if (any_l && any_r) {
            // nearer child first: order by the box centres along order_dir
            float cl = (nd.a.x + nd.a.w) * order_dir[0] + (nd.a.y + nd.b.x) * order_dir[1] +
                       (nd.a.z + nd.b.y) * order_dir[2];
            float cr = (nd.b.z + nd.c.y) * order_dir[0] + (nd.b.w + nd.c.z) * order_dir[1] +
                       (nd.c.x + nd.c.w) * order_dir[2];
            int left_first = uniform_int(cl <= cr ? 1 : 0);
            int near_ref = left_first ? ref_l : ref_r;
            int far_ref = left_first ? ref_r : ref_l;
            if (sp < kWave) {
                stack = (my_lane == sp) ? far_ref : stack;
                if (kCount) {
                    const bool far_in = left_first ? hr : hl;
                    stack_in = far_in ? (stack_in | (1ull << sp)) : (stack_in & ~(1ull << sp));
                }
                ++sp;
            } else {
                raise_flag(flags, PRTGS_FLAG_STACK_OVERFLOW);
            }
            next = near_ref;
            if (kCount) inside = left_first ? hl : hr;
        } else if (any_l) {
            next = ref_l;
            if (kCount) inside = hl;
        } else if (any_r) {
            next = ref_r;
            if (kCount) inside = hr;
        } else if (kStep == kLeavesFirst) {
            if (sp == 0) break;
            --sp;
            next = __builtin_amdgcn_readlane(stack, sp);
            if (kCount) inside = (stack_in >> sp) & 1ull;
        } else if (sp > 0) {
            --sp;
            next = __builtin_amdgcn_readlane(stack, sp);
            if (kCount) inside = (stack_in >> sp) & 1ull;
        }
        if constexpr (kStep != kLeavesFirst) {
            next = uniform_int(next);
            if (kStep == kLoadFirst && next >= 0) nd = uniform_load(nodes, next);
            if (leaf_l) {
                if (kCount && hl && live) cnt->prim_tests++;
                if (kCount) cnt->wave_leaves++;
                leaf(~ref_l, hl);
            }
            if (leaf_r) {
                if (kCount && hr && live) cnt->prim_tests++;
                if (kCount) cnt->wave_leaves++;
                leaf(~ref_r, hr);
            }
            if (next < 0 || __ballot(live) == 0ull) break;
            if (kStep == kChooseFirst) nd = uniform_load(nodes, next);
        } else {
            if (__ballot(live) == 0ull) break;
            node = next;
        }
    }
}

// ---------------------------------------------------------------------------
// Ray-Gaussian test.  With W = diag(1/s) R^T (Eq. 2: Sigma^-1 = W^T W), the
// density of Gaussian j along the ray origin + t w peaks at
// t* = -(o'.d')/(d'.d'), o' = W (origin - mu), d' = W w, with
// d^2 = |p|^2, p = W (origin - mu + t* w) (Eq. 1).  The hit test is
// t* > t_min and d^2 <= sigma_cut^2, then alpha = min(o exp(-d^2/2), alpha_max).
//
// FP32 evaluation in two stages.  The first stage forms p from o' and d'
// directly; its error (from rounding origin - mu and the products) is below
// 2e-6 (|origin - mu|_1 / s_min + 1) in whitened units, so a ray whose first-
// stage d^2 exceeds (sigma_cut + that bound)^2 cannot hit, and the second
// stage is skipped when no lane of the wave can.  The second stage builds p
// from the small world-space offset x = origin - mu + t w (FMA on the exact
// two-float difference origin - mu) and corrects it by one Newton step,
// t -= (p.d')/(d'.d'), which removes the component of p along d' that the
// error of the first t* puts there.  p, x and t* are then accurate to a few
// ulps of their own size, for d^2 and for the adjoint alike.
// ---------------------------------------------------------------------------

// a - b as an unevaluated sum s + e, exactly (Knuth's TwoSum).
__device__ inline void two_diff(float a, float b, float& s, float& e)
{
    s = a - b;
    const float bb = s - a;
    e = (a - (s - bb)) - (b + bb);
}

struct PreHit {
    float dx, dy, dz;      // origin - mu, rounded
    float e0, e1, e2, ia;  // d' = W w and 1 / (d'.d')
    float t;               // first estimate of t*
    bool maybe;            // the ray may hit (conservative)
};

__device__ inline PreHit gaussian_pre(const Prim& p, float ox, float oy, float oz, const RayDir& d, const HitParams& hp)
{
    PreHit q;
    q.dx = ox - p.mo.x;
    q.dy = oy - p.mo.y;
    q.dz = oz - p.mo.z;
    const float o0 = p.w0.x * q.dx + p.w0.y * q.dy + p.w0.z * q.dz;
    const float o1 = p.w1.x * q.dx + p.w1.y * q.dy + p.w1.z * q.dz;
    const float o2 = p.w2.x * q.dx + p.w2.y * q.dy + p.w2.z * q.dz;
    q.e0 = p.w0.x * d.wx + p.w0.y * d.wy + p.w0.z * d.wz;
    q.e1 = p.w1.x * d.wx + p.w1.y * d.wy + p.w1.z * d.wz;
    q.e2 = p.w2.x * d.wx + p.w2.y * d.wy + p.w2.z * d.wz;
    q.ia = __builtin_amdgcn_rcpf(q.e0 * q.e0 + q.e1 * q.e1 + q.e2 * q.e2);
    q.t = -(o0 * q.e0 + o1 * q.e1 + o2 * q.e2) * q.ia;
    const float p0 = fmaf(q.t, q.e0, o0), p1 = fmaf(q.t, q.e1, o1), p2 = fmaf(q.t, q.e2, o2);
    const float d2 = p0 * p0 + p1 * p1 + p2 * p2;
    const float err = 2e-6f * fmaf(fabsf(q.dx) + fabsf(q.dy) + fabsf(q.dz), p.w0.w, 1.0f);
    const float lim = hp.cut + err;
    q.maybe = d2 <= lim * lim;
    return q;
}

struct HitResult {
    float t, d2, alpha, E;   // peak position, d^2, alpha, exp(-d^2 / 2)
    float x0, x1, x2;        // origin - mu + t* w
    float p0, p1, p2;        // W (origin - mu + t* w)
};

__device__ inline bool gaussian_exact(const Prim& p, const PreHit& q, float ox, float oy, float oz, const RayDir& d,
                                      const HitParams& hp, HitResult& h)
{
    // low parts of origin - mu (TwoSum with the first stage's rounded sums)
    float bb = q.dx - ox;
    const float ex = (ox - (q.dx - bb)) - (p.mo.x + bb);
    bb = q.dy - oy;
    const float ey = (oy - (q.dy - bb)) - (p.mo.y + bb);
    bb = q.dz - oz;
    const float ez = (oz - (q.dz - bb)) - (p.mo.z + bb);
    float t = q.t;
    float x0 = fmaf(t, d.wx, q.dx) + ex;
    float x1 = fmaf(t, d.wy, q.dy) + ey;
    float x2 = fmaf(t, d.wz, q.dz) + ez;
    float p0 = p.w0.x * x0 + p.w0.y * x1 + p.w0.z * x2;
    float p1 = p.w1.x * x0 + p.w1.y * x1 + p.w1.z * x2;
    float p2 = p.w2.x * x0 + p.w2.y * x1 + p.w2.z * x2;
    const float dt = (p0 * q.e0 + p1 * q.e1 + p2 * q.e2) * q.ia;   // Newton step on t*
    t -= dt;
    x0 = fmaf(-dt, d.wx, x0);
    x1 = fmaf(-dt, d.wy, x1);
    x2 = fmaf(-dt, d.wz, x2);
    p0 = fmaf(-dt, q.e0, p0);
    p1 = fmaf(-dt, q.e1, p1);
    p2 = fmaf(-dt, q.e2, p2);
    const float d2 = p0 * p0 + p1 * p1 + p2 * p2;
    h.t = t;
    h.d2 = d2;
    h.x0 = x0; h.x1 = x1; h.x2 = x2;
    h.p0 = p0; h.p1 = p1; h.p2 = p2;
    h.E = __expf(-0.5f * d2);
    const float alpha = fminf(p.mo.w * h.E, hp.alpha_max);
    h.alpha = alpha;
    return (t > hp.t_min) & (d2 <= hp.cut2) & (alpha >= hp.alpha_min);
}

}  // namespace prtgs
