// Packet traversal of the LBVH shared by the forward, bounce and adjoint
// kernels.
//
// A wavefront traces 64 parallel rays at once: one direction w (uniform
// across the wave) from 64 different origins (the centres of 64 splats that
// are neighbours in Morton order).  The wave walks the tree together: a
// child is entered if the ray of any live lane crosses its box, so node and
// Gaussian records are read at wave-uniform addresses (scalar loads, one per
// wave instead of one per lane), the control flow never diverges, and the
// traversal stack is one VGPR -- entry k lives in lane k (a lane-select
// write, a readlane read).  Every lane still applies the exact per-ray hit test of its own
// ray at each visited Gaussian, so the result does not depend on which other
// rays share the wave.
#pragma once

#include "common.hpp"

namespace prtgs {

struct RayDir {
    float wx, wy, wz;     // direction (uniform)
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

// Interval of the ray o + t w inside the box, clipped to [tlo, thi].
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
// narrowed by `leaf`, through the references).  leaf(r) is called, uniformly,
// for every leaf rank r whose box is crossed by a live lane.  With kCount the
// lane's own single-ray work is tallied in `cnt` (the wave stack then also
// carries, per entry, the mask of lanes whose rays entered that node).
template <bool kCount = false, class LeafFn>
__device__ inline void packet_traverse(const Node* __restrict__ nodes, int n, const RayDir& d, float ox, float oy,
                                       float oz, bool& live, float& tlo, float& thi, unsigned* flags, LeafFn&& leaf,
                                       RayCounts* cnt = nullptr)
{
    if (n == 1) {
        if (__ballot(live)) {
            if (kCount && live) cnt->prim_tests++;
            if (kCount) cnt->wave_leaves++;
            leaf(0);
        }
        return;
    }
    const float oix = ox * d.ix, oiy = oy * d.iy, oiz = oz * d.iz;
    const int my_lane = __lane_id();
    int stack = 0;     // entry k of the wave's stack lives in lane k
    uint64_t stack_in = 0;   // (kCount) whether this lane's ray entered entry k's node, bit per entry
    int sp = 0;
    int node = 0;      // root
    bool inside = live;      // (kCount) this lane's ray entered the current node
    // A depth-first walk enters each of the n - 1 internal nodes at most once;
    // the cap (and the reference check) only guard against a malformed tree.
    int budget = n;
    while (true) {
        if (--budget < 0) {
            raise_flag(flags, PRTGS_FLAG_BAD_TREE);
            break;
        }
        const Node nd = uniform_load(nodes, node);
        if (kCount) cnt->wave_nodes++;
        bool hl = live && slab_hit(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, d, oix, oiy, oiz, tlo, thi);
        bool hr = live && slab_hit(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, d, oix, oiy, oiz, tlo, thi);
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
        if (any_l && ref_l < 0) {
            if (kCount && hl && live) cnt->prim_tests++;
            if (kCount) cnt->wave_leaves++;
            leaf(~ref_l);
            any_l = false;
        }
        if (any_r && ref_r < 0) {
            if (kCount && hr && live) cnt->prim_tests++;
            if (kCount) cnt->wave_leaves++;
            leaf(~ref_r);
            any_r = false;
        }
        int next;
        if (any_l && any_r) {
            // nearer child first: order by the box centres along w
            float cl = (nd.a.x + nd.a.w) * d.wx + (nd.a.y + nd.b.x) * d.wy + (nd.a.z + nd.b.y) * d.wz;
            float cr = (nd.b.z + nd.c.y) * d.wx + (nd.b.w + nd.c.z) * d.wy + (nd.c.x + nd.c.w) * d.wz;
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
        } else {
            if (sp == 0) break;
            --sp;
            next = __builtin_amdgcn_readlane(stack, sp);
            if (kCount) inside = (stack_in >> sp) & 1ull;
        }
        if (__ballot(live) == 0ull) break;
        node = next;
    }
}

// a - b as an unevaluated sum s + e, exactly (Knuth's TwoSum).
__device__ inline void two_diff(float a, float b, float& s, float& e)
{
    s = a - b;
    const float bb = s - a;
    e = (a - (s - bb)) - (b + bb);
}

// Exact per-ray test of one Gaussian (record p) for the ray origin.  With
// W = diag(1/s) R^T (Eq. 2: Sigma^-1 = W^T W), the density along the ray
// peaks at t* = -(o'.d')/(d'.d'), o' = W (origin - mu), d' = W w, and
// d^2 = |p|^2 with p = W (origin - mu + t* w) there (Eq. 1).
// Evaluation in FP32: the first estimate of t* carries an error of order
// eps |origin - mu| / s_min for thin, distant Gaussians.  p is therefore
// built from the small world-space offset x = origin - mu + t w (FMA on the
// exact two-float difference origin - mu) and then corrected by one Newton
// step, t -= (p.d')/(d'.d'), which removes the component of p along d' that
// the error in t puts there.  Then p, x and t* are accurate to a few ulps of
// their own (small) size, for d^2 and for the adjoint alike.
struct HitResult {
    float t, d2, alpha, E;   // peak position, d^2, alpha, exp(-d^2 / 2)
    float x0, x1, x2;        // origin - mu + t* w
    float p0, p1, p2;        // W (origin - mu + t* w)
};

__device__ inline bool gaussian_hit(const Prim& p, float ox, float oy, float oz, const RayDir& d, const HitParams& hp,
                                    HitResult& h)
{
    float dx, dy, dz, ex, ey, ez;
    two_diff(ox, p.mo.x, dx, ex);
    two_diff(oy, p.mo.y, dy, ey);
    two_diff(oz, p.mo.z, dz, ez);
    const float o0 = p.w0.x * dx + p.w0.y * dy + p.w0.z * dz;
    const float o1 = p.w1.x * dx + p.w1.y * dy + p.w1.z * dz;
    const float o2 = p.w2.x * dx + p.w2.y * dy + p.w2.z * dz;
    const float e0 = p.w0.x * d.wx + p.w0.y * d.wy + p.w0.z * d.wz;
    const float e1 = p.w1.x * d.wx + p.w1.y * d.wy + p.w1.z * d.wz;
    const float e2 = p.w2.x * d.wx + p.w2.y * d.wy + p.w2.z * d.wz;
    const float ia = __builtin_amdgcn_rcpf(e0 * e0 + e1 * e1 + e2 * e2);
    float t = -(o0 * e0 + o1 * e1 + o2 * e2) * ia;
    float x0 = fmaf(t, d.wx, dx) + ex;
    float x1 = fmaf(t, d.wy, dy) + ey;
    float x2 = fmaf(t, d.wz, dz) + ez;
    float p0 = p.w0.x * x0 + p.w0.y * x1 + p.w0.z * x2;
    float p1 = p.w1.x * x0 + p.w1.y * x1 + p.w1.z * x2;
    float p2 = p.w2.x * x0 + p.w2.y * x1 + p.w2.z * x2;
    const float dt = (p0 * e0 + p1 * e1 + p2 * e2) * ia;   // Newton step on t*
    t -= dt;
    x0 = fmaf(-dt, d.wx, x0);
    x1 = fmaf(-dt, d.wy, x1);
    x2 = fmaf(-dt, d.wz, x2);
    p0 = fmaf(-dt, e0, p0);
    p1 = fmaf(-dt, e1, p1);
    p2 = fmaf(-dt, e2, p2);
    const float d2 = p0 * p0 + p1 * p1 + p2 * p2;
    h.t = t;
    h.d2 = d2;
    h.x0 = x0; h.x1 = x1; h.x2 = x2;
    h.p0 = p0; h.p1 = p1; h.p2 = p2;
    if (!(t > hp.t_min) || !(d2 <= hp.cut2)) return false;
    h.E = __expf(-0.5f * d2);
    const float alpha = fminf(p.mo.w * h.E, hp.alpha_max);
    h.alpha = alpha;
    return alpha >= hp.alpha_min;
}

}  // namespace prtgs
