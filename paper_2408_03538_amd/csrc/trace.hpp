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

// Walks the BVH for the wave's rays.  `live` is the lane's participation
// (may be cleared by `leaf`), [tlo, thi] the lane's ray interval (may be
// narrowed by `leaf`, through the references).  leaf(r) is called, uniformly,
// for every leaf rank r whose box is crossed by a live lane.
template <class LeafFn>
__device__ inline void packet_traverse(const Node* __restrict__ nodes, int n, const RayDir& d, float ox, float oy,
                                       float oz, bool& live, float& tlo, float& thi, unsigned* flags, LeafFn&& leaf)
{
    if (n == 1) {
        if (__ballot(live)) leaf(0);
        return;
    }
    const float oix = ox * d.ix, oiy = oy * d.iy, oiz = oz * d.iz;
    const int my_lane = __lane_id();
    int stack = 0;     // entry k of the wave's stack lives in lane k
    int sp = 0;
    int node = 0;      // root
    // A depth-first walk enters each of the n - 1 internal nodes at most once;
    // the cap (and the reference check) only guard against a malformed tree.
    int budget = n;
    while (true) {
        if (--budget < 0) {
            raise_flag(flags, PRTGS_FLAG_BAD_TREE);
            break;
        }
        const Node nd = uniform_load(nodes, node);
        bool hl = live && slab_hit(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, d, oix, oiy, oiz, tlo, thi);
        bool hr = live && slab_hit(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, d, oix, oiy, oiz, tlo, thi);
        bool any_l = __ballot(hl) != 0ull;
        bool any_r = __ballot(hr) != 0ull;
        const int ref_l = nd.d.x, ref_r = nd.d.y;
        if (ref_l >= n - 1 || ~ref_l >= n || ref_r >= n - 1 || ~ref_r >= n) {
            raise_flag(flags, PRTGS_FLAG_BAD_TREE);
            break;
        }
        if (any_l && ref_l < 0) {
            leaf(~ref_l);
            any_l = false;
        }
        if (any_r && ref_r < 0) {
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
                ++sp;
            } else {
                raise_flag(flags, PRTGS_FLAG_STACK_OVERFLOW);
            }
            next = near_ref;
        } else if (any_l) {
            next = ref_l;
        } else if (any_r) {
            next = ref_r;
        } else {
            if (sp == 0) break;
            --sp;
            next = __builtin_amdgcn_readlane(stack, sp);
        }
        if (__ballot(live) == 0ull) break;
        node = next;
    }
}

// Exact per-ray test of one Gaussian (record p) for the ray origin - the
// whitened form: with W = diag(1/s) R^T, o' = W (origin - mu) and d' = W w,
// the density along the ray peaks at t* = -(o'.d')/(d'.d') and
// d^2 = |o' + t* d'|^2 there (Eq. 1-2).  Returns whether it is a hit.
struct HitResult {
    float t, d2, alpha;
};

__device__ inline bool gaussian_hit(const Prim& p, float ox, float oy, float oz, const RayDir& d, const HitParams& hp,
                                    HitResult& h)
{
    float dx = ox - p.mo.x, dy = oy - p.mo.y, dz = oz - p.mo.z;
    float o0 = p.w0.x * dx + p.w0.y * dy + p.w0.z * dz;
    float o1 = p.w1.x * dx + p.w1.y * dy + p.w1.z * dz;
    float o2 = p.w2.x * dx + p.w2.y * dy + p.w2.z * dz;
    float e0 = p.w0.x * d.wx + p.w0.y * d.wy + p.w0.z * d.wz;
    float e1 = p.w1.x * d.wx + p.w1.y * d.wy + p.w1.z * d.wz;
    float e2 = p.w2.x * d.wx + p.w2.y * d.wy + p.w2.z * d.wz;
    float a = e0 * e0 + e1 * e1 + e2 * e2;
    float b = o0 * e0 + o1 * e1 + o2 * e2;
    float t = -b * __builtin_amdgcn_rcpf(a);
    float p0 = fmaf(t, e0, o0), p1 = fmaf(t, e1, o1), p2 = fmaf(t, e2, o2);
    float d2 = p0 * p0 + p1 * p1 + p2 * p2;
    h.t = t;
    h.d2 = d2;
    if (!(t > hp.t_min) || !(d2 <= hp.cut2)) return false;
    float alpha = fminf(p.mo.w * __expf(-0.5f * d2), hp.alpha_max);
    h.alpha = alpha;
    return alpha >= hp.alpha_min;
}

}  // namespace prtgs
