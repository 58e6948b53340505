// C ABI of the library: host-side validation, workspace carving and dispatch
// to the kernels.  No device memory is allocated here.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "common.hpp"

namespace prtgs {

void stratified_grid(int S, int* nu, int* nv);

namespace {

thread_local char g_err[512] = "";

prtgs_status fail(prtgs_status s, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

prtgs_status ok()
{
    g_err[0] = '\0';
    return PRTGS_OK;
}

prtgs_status hip_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return ok();
    return fail(PRTGS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

constexpr int kMaxN = 1 << 30;

prtgs_status check_gaussians(const prtgs_gaussians* g, bool need_albedo)
{
    if (!g) return fail(PRTGS_ERR_INVALID_ARG, "gaussians struct is NULL");
    if (g->n < 1 || g->n > kMaxN) return fail(PRTGS_ERR_INVALID_ARG, "n = %d outside [1, 2^30]", g->n);
    if (!g->means || !g->quats || !g->log_scales || !g->opacity || !g->normals)
        return fail(PRTGS_ERR_INVALID_ARG, "a Gaussian attribute pointer is NULL");
    if (need_albedo && !g->albedo) return fail(PRTGS_ERR_INVALID_ARG, "albedo is NULL but a bounce was requested");
    return PRTGS_OK;
}

prtgs_status check_desc(const prtgs_transfer_desc* d)
{
    if (!d) return fail(PRTGS_ERR_INVALID_ARG, "transfer desc is NULL");
    if (d->num_dirs < 1 || d->num_dirs > 65536)
        return fail(PRTGS_ERR_INVALID_ARG, "num_dirs = %d outside [1, 65536]", d->num_dirs);
    if (d->sh_bands < 1 || d->sh_bands > 4)
        return fail(PRTGS_ERR_INVALID_ARG, "sh_bands = %d outside [1, 4]", d->sh_bands);
    if (d->bounce_mode != PRTGS_BOUNCE_BLEND && d->bounce_mode != PRTGS_BOUNCE_INDEX)
        return fail(PRTGS_ERR_INVALID_ARG, "bounce_mode = %d unknown", d->bounce_mode);
    if (d->bounce_mode == PRTGS_BOUNCE_BLEND && d->bounces != 0 && d->bounces != 1)
        return fail(PRTGS_ERR_INVALID_ARG, "bounces = %d: the blended bounce takes 0 or 1", d->bounces);
    if (d->bounce_mode == PRTGS_BOUNCE_INDEX && (d->bounces < 0 || d->bounces > PRTGS_MAX_INDEX_BOUNCES))
        return fail(PRTGS_ERR_INVALID_ARG, "bounces = %d outside [0, %d]", d->bounces, PRTGS_MAX_INDEX_BOUNCES);
    if (!(d->t_same > 0.0f && d->t_same <= 1.0f)) return fail(PRTGS_ERR_INVALID_ARG, "t_same outside (0, 1]");
    if (!(d->sigma_cut > 0.0f && d->sigma_cut <= kBoxSigma))
        return fail(PRTGS_ERR_INVALID_ARG, "sigma_cut = %g outside (0, 3] (BVH boxes are 3-sigma)", d->sigma_cut);
    if (!std::isfinite(d->t_min) || d->t_min < 0.0f) return fail(PRTGS_ERR_INVALID_ARG, "t_min must be finite and >= 0");
    if (!(d->T_eps >= 0.0f && d->T_eps < 1.0f)) return fail(PRTGS_ERR_INVALID_ARG, "T_eps outside [0, 1)");
    if (!(d->alpha_max > 0.0f && d->alpha_max <= 0.999f))
        return fail(PRTGS_ERR_INVALID_ARG, "alpha_max outside (0, 0.999]");
    if (!(d->alpha_min >= 0.0f && d->alpha_min <= d->alpha_max))
        return fail(PRTGS_ERR_INVALID_ARG, "alpha_min outside [0, alpha_max]");
    const int g = d->sources_per_wave;
    if (g != 0 && g != 1 && g != 2 && g != 4 && g != 8 && g != 16 && g != 32 && g != 64)
        return fail(PRTGS_ERR_INVALID_ARG, "sources_per_wave = %d not 0 or a power of two up to 64", g);
    if (d->direction_parts < 0 || d->direction_parts > 64)
        return fail(PRTGS_ERR_INVALID_ARG, "direction_parts = %d outside [0, 64]", d->direction_parts);
    if (d->bounce_records < 0 || d->bounce_records > ((int64_t)1 << 40))
        return fail(PRTGS_ERR_INVALID_ARG, "bounce_records = %lld outside [0, 2^40]", (long long)d->bounce_records);
    return PRTGS_OK;
}

// The blended bounce runs as one walk per ray when the caller gives it a record arena.
bool one_walk(const prtgs_transfer_desc& d)
{
    return d.bounces == 1 && d.bounce_mode == PRTGS_BOUNCE_BLEND && d.bounce_records > 0;
}
// So does the index matrix, on the same switch (it keeps no records: no arena).
bool one_walk_index(const prtgs_transfer_desc& d)
{
    return d.bounces >= 1 && d.bounce_mode == PRTGS_BOUNCE_INDEX && d.bounce_records > 0;
}

// Sources per wave of the group split; 1 selects the fan kernel.  With the
// direction batches spread over waves a launch holds ~count S / 64 waves
// whatever G is, so the default is chosen by measurement (S = 256 surface
// scenes): 16 from 40k sources (50k: 6.2 ms against 6.7 for G = 8; 100k: 16.9
// against 19.5), 8 from 10k (20k: 1.9 against 2.0 for 16, 2.9 for 2), 4 from
// 2048 (5k: 0.61 against 0.89 for the fan kernel), the fan kernel below.
// `requested` (a power of two up to 64, 0 = this default) is the caller's.
int group_size(int count, int requested)
{
    if (requested > 0) return requested;
    return count >= 40000 ? 16 : count >= 10000 ? 8 : count >= 2048 ? 4 : 1;
}

// The blend's buffers: its direction parts (each with a [n][3][K] set of
// sums) and, for one walk, its work items (part, source group).  A bounce
// covers the whole scene (first = 0, count = n), so the launch takes its
// group size from n as this does.
struct BlendNeed {
    int parts;
    int64_t items;
};

BlendNeed blend_need(const prtgs_transfer_desc& d, int n)
{
    const int G = group_size(n, d.sources_per_wave);
    const int Q = blend_parts(G, d.num_dirs, d.direction_parts);
    return {Q, (int64_t)((n + G - 1) / G) * Q};
}

struct TransferWs {
    size_t dirs, Y, dir_order, rayw, hits, tcut, queue, hitkey, hitalpha, hitrec, partial, index, term0, term1,
        rec_top, item_head, item_deferred, rec, total;
    int64_t items;   // one-walk blend: work items (direction part, source group)
};

TransferWs transfer_ws_layout(const prtgs_transfer_desc& d, int n)
{
    TransferWs w;
    int K = d.sh_bands * d.sh_bands;
    size_t off = kFlagBytes;
    w.dirs = off;
    off += align256(sizeof(float) * 3 * (size_t)d.num_dirs);
    w.Y = off;
    off += align256(sizeof(float) * (size_t)K * (size_t)d.num_dirs);
    w.dir_order = off;
    off += align256(sizeof(int32_t) * (size_t)d.num_dirs);
    w.rayw = off;
    off += align256(sizeof(float) * (size_t)n * (size_t)d.num_dirs);
    w.hits = off;
    if (d.bounces) off += align256(sizeof(float) * (size_t)hit_stride(K) * (size_t)n);
    w.tcut = off;
    if (d.bounces) off += align256(sizeof(float) * (size_t)n * (size_t)d.num_dirs);
    w.queue = off;
    if (d.bounces) off += 256;
    // index mode: the index matrix and two bounce terms [n][3][K] (ping-pong)
    const bool idx = d.bounces && d.bounce_mode == PRTGS_BOUNCE_INDEX;
    // the lists hold the persistent waves of every walk the call may run (one walk: its own and the two-walk
    // pass over deferred items)
    const size_t lw = idx ? bounce_waves(n, kWalkIndex)
                          : std::max(bounce_waves(n, kWalkBlend), one_walk(d) ? bounce_waves(n, kWalkFused) : 0);
    w.hitkey = off;
    if (d.bounces) off += align256(lw * kHitList * 64 * 8);
    w.hitalpha = off;
    if (d.bounces) off += align256(lw * kHitList * 64 * 4);
    w.hitrec = off;
    if (d.bounces && !idx) off += align256(lw * kHitList * 64 * 8);
    const BlendNeed need = d.bounces && !idx ? blend_need(d, n) : BlendNeed{0, 0};
    w.partial = off;
    off += align256(sizeof(float) * need.parts * 3 * (size_t)K * (size_t)n);
    w.index = off;
    if (idx) off += align256(sizeof(int32_t) * (size_t)n * (size_t)d.num_dirs);
    w.term0 = off;
    if (idx) off += align256(sizeof(float) * 3 * (size_t)K * (size_t)n);
    w.term1 = off;
    if (idx) off += align256(sizeof(float) * 3 * (size_t)K * (size_t)n);
    // one-walk blend: the record arena and per work item its first block and deferral mark
    const bool fused = one_walk(d);
    w.items = fused ? need.items : 0;
    w.rec_top = off;
    if (fused) off += 256;
    w.item_head = off;
    off += align256(sizeof(int64_t) * (size_t)w.items);
    w.item_deferred = off;
    off += align256(sizeof(int32_t) * (size_t)w.items);
    w.rec = off;
    if (fused) off += align256(8 * (size_t)d.bounce_records);
    w.total = off;
    return w;
}

HitParams hit_params(const prtgs_transfer_desc& d)
{
    HitParams h;
    h.cut = d.sigma_cut;
    h.cut2 = d.sigma_cut * d.sigma_cut;
    h.t_min = d.t_min;
    h.T_eps = d.T_eps;
    h.alpha_min = d.alpha_min;
    h.alpha_max = d.alpha_max;
    return h;
}

}  // namespace
}  // namespace prtgs

using namespace prtgs;

extern "C" {

int32_t prtgs_abi_version(void) { return PRTGS_ABI_VERSION; }

const char* prtgs_last_error(void) { return g_err; }

const char* prtgs_status_string(prtgs_status s)
{
    switch (s) {
        case PRTGS_OK: return "ok";
        case PRTGS_ERR_INVALID_ARG: return "invalid argument";
        case PRTGS_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case PRTGS_ERR_UNSUPPORTED: return "unsupported";
        case PRTGS_ERR_HIP: return "HIP error";
    }
    return "unknown status";
}

prtgs_status prtgs_direction_table(int32_t num_dirs, uint64_t seed, int32_t sh_bands, double* dirs64, double* Y64,
                                   float* dirs32, float* Y32, hipStream_t stream)
{
    if (num_dirs < 1 || num_dirs > 65536) return fail(PRTGS_ERR_INVALID_ARG, "num_dirs = %d outside [1, 65536]", num_dirs);
    if (sh_bands < 1 || sh_bands > 8) return fail(PRTGS_ERR_INVALID_ARG, "sh_bands = %d outside [1, 8]", sh_bands);
    if (!dirs64 && !Y64 && !dirs32 && !Y32) return ok();
    return hip_status(launch_direction_table(num_dirs, seed, sh_bands, dirs64, Y64, dirs32, Y32, stream),
                      "direction table");
}

size_t prtgs_bvh_bytes(int32_t n) { return n < 1 ? 0 : bvh_layout(n).total; }

size_t prtgs_build_workspace_bytes(int32_t n) { return n < 1 ? 0 : build_workspace_bytes(n); }

prtgs_status prtgs_build_bvh(const prtgs_gaussians* g, void* bvh, size_t bvh_bytes, void* ws, size_t ws_bytes,
                             hipStream_t stream)
{
    prtgs_status st = check_gaussians(g, false);
    if (st != PRTGS_OK) return st;
    if (!bvh || !ws) return fail(PRTGS_ERR_INVALID_ARG, "bvh or workspace is NULL");
    if (!aligned256(bvh) || !aligned256(ws)) return fail(PRTGS_ERR_INVALID_ARG, "bvh and workspace must be 256-byte aligned");
    if (bvh_bytes < prtgs_bvh_bytes(g->n))
        return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "bvh buffer has %zu bytes, needs %zu", bvh_bytes, prtgs_bvh_bytes(g->n));
    if (ws_bytes < prtgs_build_workspace_bytes(g->n))
        return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes,
                    prtgs_build_workspace_bytes(g->n));
    unsigned* flags = static_cast<unsigned*>(ws);
    hipError_t e = fill_u32(flags, 0u, 1, stream);
    if (e == hipSuccess) e = launch_build_bvh(*g, bvh, ws, flags, stream);
    return hip_status(e, "build bvh");
}

prtgs_status prtgs_bvh_leaf_order(const void* bvh, int32_t n, int32_t* order, hipStream_t stream)
{
    if (!bvh || !order) return fail(PRTGS_ERR_INVALID_ARG, "bvh or order is NULL");
    if (n < 1 || n > kMaxN) return fail(PRTGS_ERR_INVALID_ARG, "n = %d outside [1, 2^30]", n);
    return hip_status(launch_leaf_order(bvh, n, order, stream), "leaf order copy");
}

size_t prtgs_transfer_workspace_bytes(const prtgs_transfer_desc* d, int32_t n)
{
    if (!d || n < 1 || check_desc(d) != PRTGS_OK) return 0;
    return transfer_ws_layout(*d, n).total;
}

}  // extern "C"

namespace {

// Arguments of the transfer kernels for sources [first, first + count).
TransferArgs transfer_args(const prtgs_gaussians* g, const void* bvh, const prtgs_transfer_desc* d, int first,
                           int count, float* transfer, float* vis, char* w, const TransferWs& W)
{
    const int n = g->n;
    const BvhLayout L = bvh_layout(n);
    const char* b = static_cast<const char*>(bvh);
    const bool bounce = d->bounces > 0;
    TransferArgs a{};
    a.nodes = reinterpret_cast<const Node*>(b + L.nodes);
    a.prims = reinterpret_cast<const Prim*>(b + L.prims);
    a.normals = reinterpret_cast<const float4*>(b + L.normals);
    a.order = reinterpret_cast<const int32_t*>(b + L.order);
    a.dirs = reinterpret_cast<const float*>(w + W.dirs);
    a.Y = reinterpret_cast<const float*>(w + W.Y);
    a.dir_order = reinterpret_cast<const int32_t*>(w + W.dir_order);
    a.S = d->num_dirs;
    a.K = d->sh_bands * d->sh_bands;
    a.n = n;
    a.first = first;
    a.count = count;
    a.channels = bounce ? 3 : 1;
    a.hp = hit_params(*d);
    a.transfer = transfer;
    a.vis = vis;
    a.hit_table = bounce ? reinterpret_cast<float*>(w + W.hits) : nullptr;
    a.albedo = g->albedo;
    a.rayw = reinterpret_cast<float*>(w + W.rayw);
    a.tcut = bounce ? reinterpret_cast<float*>(w + W.tcut) : nullptr;
    a.queue = bounce ? reinterpret_cast<unsigned*>(w + W.queue) : nullptr;
    a.hitkey = bounce ? reinterpret_cast<uint64_t*>(w + W.hitkey) : nullptr;
    a.hitalpha = bounce ? reinterpret_cast<float*>(w + W.hitalpha) : nullptr;
    a.hitrec = bounce && d->bounce_mode == PRTGS_BOUNCE_BLEND ? reinterpret_cast<int2*>(w + W.hitrec) : nullptr;
    a.partial = bounce && d->bounce_mode == PRTGS_BOUNCE_BLEND ? reinterpret_cast<float*>(w + W.partial) : nullptr;
    a.index = nullptr;
    a.t_same = d->t_same;
    a.G = group_size(count, d->sources_per_wave);
    a.Q_req = d->direction_parts;
    a.flags = reinterpret_cast<unsigned*>(w);
    if (one_walk(*d)) {
        a.rec = reinterpret_cast<uint64_t*>(w + W.rec);
        a.rec_words = (uint64_t)d->bounce_records;
        a.rec_top = reinterpret_cast<unsigned long long*>(w + W.rec_top);
        a.item_head = reinterpret_cast<int64_t*>(w + W.item_head);
        a.item_deferred = reinterpret_cast<int32_t*>(w + W.item_deferred);
    }
    return a;
}

// Flag word cleared, direction and SH tables and the direction order built.
hipError_t transfer_setup(const prtgs_transfer_desc* d, char* w, const TransferWs& W, hipStream_t stream)
{
    hipError_t e = fill_u32(reinterpret_cast<unsigned*>(w), 0u, 1, stream);
    if (e == hipSuccess)
        e = launch_direction_table(d->num_dirs, d->seed, d->sh_bands, nullptr, nullptr,
                                   reinterpret_cast<float*>(w + W.dirs), reinterpret_cast<float*>(w + W.Y), stream);
    if (e == hipSuccess) e = launch_direction_order(d->num_dirs, reinterpret_cast<int32_t*>(w + W.dir_order), stream);
    return e;
}

}  // namespace

extern "C" {

prtgs_status prtgs_precompute_transfer(const prtgs_gaussians* g, const void* bvh, const prtgs_transfer_desc* d,
                                       int32_t first, int32_t count, float* transfer, float* vis, void* ws,
                                       size_t ws_bytes, hipStream_t stream)
{
    prtgs_status st = check_desc(d);
    if (st != PRTGS_OK) return st;
    st = check_gaussians(g, d->bounces > 0);
    if (st != PRTGS_OK) return st;
    const int n = g->n;
    if (!bvh || !ws) return fail(PRTGS_ERR_INVALID_ARG, "bvh or workspace is NULL");
    if (!aligned256(bvh) || !aligned256(ws)) return fail(PRTGS_ERR_INVALID_ARG, "bvh and workspace must be 256-byte aligned");
    if (first < 0 || count < 0 || (int64_t)first + count > n)
        return fail(PRTGS_ERR_INVALID_ARG, "source range [%d, %d + %d) outside [0, %d)", first, first, count, n);
    if (d->bounces > 0 && (first != 0 || count != n))
        return fail(PRTGS_ERR_INVALID_ARG, "a bounce needs every source's direct transfer: use first = 0, count = n");
    if (count > 0 && !transfer) return fail(PRTGS_ERR_INVALID_ARG, "transfer is NULL");
    TransferWs W = transfer_ws_layout(*d, n);
    if (ws_bytes < W.total)
        return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes, W.total);

    char* w = static_cast<char*>(ws);
    hipError_t e = transfer_setup(d, w, W, stream);
    if (e != hipSuccess) return hip_status(e, "direction table");
    if (count == 0) return ok();
    TransferArgs a = transfer_args(g, bvh, d, first, count, transfer, vis, w, W);
    if (one_walk(*d)) return hip_status(launch_transfer_fused(a, stream), "one-walk blended bounce");
    if (one_walk_index(*d)) {
        a.index = reinterpret_cast<int32_t*>(w + W.index);
        e = launch_index_fused(a, stream, true);
        if (e != hipSuccess) return hip_status(e, "one-walk index matrix");
    } else {
        e = launch_transfer_direct(a, stream);
        if (e != hipSuccess) return hip_status(e, "direct transfer");
        if (d->bounces > 0 && d->bounce_mode == PRTGS_BOUNCE_BLEND) {
            e = launch_transfer_bounce(a, stream);
            if (e != hipSuccess) return hip_status(e, "bounce transfer");
        } else if (d->bounces > 0) {
            a.index = reinterpret_cast<int32_t*>(w + W.index);
            e = launch_transfer_index(a, stream);
            if (e != hipSuccess) return hip_status(e, "index matrix");
        }
    }
    if (d->bounces > 0 && d->bounce_mode == PRTGS_BOUNCE_INDEX) {
        // T^m from T^(m-1) by gathers; T^0 is the direct transfer the output
        // already holds in all three channels
        const int K = a.K;
        float* terms[2] = {reinterpret_cast<float*>(w + W.term0), reinterpret_cast<float*>(w + W.term1)};
        const float* prev = transfer;
        for (int m = 1; m <= d->bounces; ++m) {
            float* out = terms[(m - 1) % 2];
            e = launch_self_transfer(n, a.S, K, a.dirs, g->normals, g->albedo, a.index, prev, 3, out, a.flags, stream);
            if (e == hipSuccess) e = launch_add(transfer, out, (size_t)n * 3 * K, stream);
            if (e != hipSuccess) return hip_status(e, "self-transfer");
            prev = out;
        }
    }
    return ok();
}

prtgs_status prtgs_index_matrix(const prtgs_gaussians* g, const void* bvh, const prtgs_transfer_desc* d,
                                int32_t* index, void* ws, size_t ws_bytes, hipStream_t stream)
{
    prtgs_status st = check_desc(d);
    if (st != PRTGS_OK) return st;
    st = check_gaussians(g, false);
    if (st != PRTGS_OK) return st;
    const int n = g->n;
    if (!bvh || !ws || !index) return fail(PRTGS_ERR_INVALID_ARG, "bvh, index or workspace is NULL");
    if (!aligned256(bvh) || !aligned256(ws)) return fail(PRTGS_ERR_INVALID_ARG, "bvh and workspace must be 256-byte aligned");
    // the workspace of the index mode with at least one bounce
    prtgs_transfer_desc di = *d;
    di.bounce_mode = PRTGS_BOUNCE_INDEX;
    if (di.bounces < 1) di.bounces = 1;
    TransferWs W = transfer_ws_layout(di, n);
    if (ws_bytes < W.total)
        return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes, W.total);
    char* w = static_cast<char*>(ws);
    hipError_t e = transfer_setup(&di, w, W, stream);
    if (e != hipSuccess) return hip_status(e, "direction table");
    // direct pass into scratch (its per-ray depths bound the walk), then the walk
    TransferArgs a = transfer_args(g, bvh, &di, 0, n, reinterpret_cast<float*>(w + W.term0), nullptr, w, W);
    a.channels = 1;
    a.hit_table = nullptr;   // the walk needs neither the sorted transfers nor the albedo
    a.albedo = nullptr;
    a.index = index;
    // one walk: the index matrix with the visibility (into scratch), no projection
    if (one_walk_index(di)) return hip_status(launch_index_fused(a, stream, false), "one-walk index matrix");
    e = launch_transfer_direct(a, stream);
    if (e != hipSuccess) return hip_status(e, "direct transfer");
    return hip_status(launch_transfer_index(a, stream), "index matrix");
}

prtgs_status prtgs_self_transfer(int32_t n, int32_t S, int32_t K, const float* dirs, const float* normals,
                                 const float* albedo, const int32_t* index, const float* t_prev, int32_t c_prev,
                                 float* t_out, unsigned* flags, hipStream_t stream)
{
    if (n < 0) return fail(PRTGS_ERR_INVALID_ARG, "n < 0");
    if (S < 1 || S > 65536) return fail(PRTGS_ERR_INVALID_ARG, "S = %d outside [1, 65536]", S);
    if (K != 1 && K != 4 && K != 9 && K != 16) return fail(PRTGS_ERR_INVALID_ARG, "K = %d not 1, 4, 9 or 16", K);
    if (c_prev != 1 && c_prev != 3) return fail(PRTGS_ERR_INVALID_ARG, "c_prev = %d not 1 or 3", c_prev);
    if (n == 0) return ok();
    if (!dirs || !normals || !albedo || !index || !t_prev || !t_out)
        return fail(PRTGS_ERR_INVALID_ARG, "a self-transfer pointer is NULL");
    if (t_out == t_prev) return fail(PRTGS_ERR_INVALID_ARG, "t_out must not alias t_prev");
    return hip_status(launch_self_transfer(n, S, K, dirs, normals, albedo, index, t_prev, c_prev, t_out, flags, stream),
                      "self-transfer");
}

}  // extern "C"

namespace {

struct SplatWs {
    size_t uv, conic_o, depth, rect, count, offset, total, ranges, keys, keys_alt, vals, vals_alt, scan, sort, end;
    size_t scan_bytes, sort_bytes;
};

bool splat_ws_layout(int n, int width, int height, int64_t max_instances, SplatWs& w)
{
    const size_t ntiles = (size_t)((width + 15) / 16) * (size_t)((height + 15) / 16);
    w.scan_bytes = splat_scan_temp_bytes(n);
    w.sort_bytes = splat_sort_temp_bytes(max_instances > 0 ? max_instances : 1);
    if (w.scan_bytes == 0 || w.sort_bytes == 0) return false;
    size_t off = kFlagBytes;
    auto take = [&](size_t& at, size_t bytes) {
        at = off;
        off += align256(bytes);
    };
    take(w.uv, 16 * (size_t)n);
    take(w.conic_o, 16 * (size_t)n);
    take(w.depth, 4 * (size_t)n);
    take(w.rect, 16 * (size_t)n);
    take(w.count, 4 * (size_t)n);
    take(w.offset, 8 * (size_t)n);
    take(w.total, 8);
    take(w.ranges, 8 * ntiles);
    take(w.keys, 8 * (size_t)max_instances);
    take(w.keys_alt, 8 * (size_t)max_instances);
    take(w.vals, 4 * (size_t)max_instances);
    take(w.vals_alt, 4 * (size_t)max_instances);
    take(w.scan, w.scan_bytes);
    take(w.sort, w.sort_bytes);
    w.end = off;
    return true;
}

prtgs_status check_camera(const prtgs_camera* c)
{
    if (!c) return fail(PRTGS_ERR_INVALID_ARG, "camera is NULL");
    if (c->width < 1 || c->width > 16384 || c->height < 1 || c->height > 16384)
        return fail(PRTGS_ERR_INVALID_ARG, "image %d x %d outside [1, 16384]^2", c->width, c->height);
    if (!(c->near_z > 0.0f) || !std::isfinite(c->near_z)) return fail(PRTGS_ERR_INVALID_ARG, "near_z must be > 0");
    if (!(c->fx > 0.0f && c->fy > 0.0f) || !std::isfinite(c->fx) || !std::isfinite(c->fy) || !std::isfinite(c->cx) ||
        !std::isfinite(c->cy))
        return fail(PRTGS_ERR_INVALID_ARG, "intrinsics must be finite with fx, fy > 0");
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(c->view[i])) return fail(PRTGS_ERR_INVALID_ARG, "view matrix is not finite");
    return PRTGS_OK;
}

}  // namespace

extern "C" {

size_t prtgs_splat_workspace_bytes(int32_t n, int32_t width, int32_t height, int64_t max_instances)
{
    if (n < 1 || width < 1 || height < 1 || width > 16384 || height > 16384 || max_instances < 0 ||
        max_instances > (int64_t)UINT32_MAX)
        return 0;
    SplatWs w;
    if (!splat_ws_layout(n, width, height, max_instances, w)) return 0;
    return w.end;
}

prtgs_status prtgs_splat_render(const prtgs_gaussians* g, const float* colours, int64_t colour_stride,
                                const prtgs_camera* cam, float* image, float* final_T, int64_t max_instances,
                                void* ws, size_t ws_bytes, int64_t* instances, hipStream_t stream)
{
    prtgs_status st = check_gaussians(g, false);
    if (st != PRTGS_OK) return st;
    st = check_camera(cam);
    if (st != PRTGS_OK) return st;
    if (!colours || !image || !ws) return fail(PRTGS_ERR_INVALID_ARG, "colours, image or workspace is NULL");
    if (colour_stride < 3) return fail(PRTGS_ERR_INVALID_ARG, "colour_stride < 3");
    if (!aligned256(ws)) return fail(PRTGS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (max_instances < 0 || max_instances > (int64_t)UINT32_MAX)
        return fail(PRTGS_ERR_INVALID_ARG, "max_instances outside [0, 2^32)");
    const int n = g->n;
    SplatWs W;
    if (!splat_ws_layout(n, cam->width, cam->height, max_instances, W))
        return fail(PRTGS_ERR_HIP, "sort / scan size query failed");
    if (ws_bytes < W.end)
        return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes, W.end);
    char* w = static_cast<char*>(ws);
    SplatCamera c;
    for (int i = 0; i < 12; ++i) c.view[i] = cam->view[i];
    c.fx = cam->fx;
    c.fy = cam->fy;
    c.cx = cam->cx;
    c.cy = cam->cy;
    c.width = cam->width;
    c.height = cam->height;
    c.near_z = cam->near_z;
    for (int i = 0; i < 3; ++i) c.background[i] = cam->background[i];
    c.lim[0] = -1.3f * cam->cx / cam->fx;
    c.lim[1] = 1.3f * ((float)cam->width - cam->cx) / cam->fx;
    c.lim[2] = -1.3f * cam->cy / cam->fy;
    c.lim[3] = 1.3f * ((float)cam->height - cam->cy) / cam->fy;
    SplatBuffers b;
    b.uv = reinterpret_cast<float4*>(w + W.uv);
    b.conic_o = reinterpret_cast<float4*>(w + W.conic_o);
    b.depth = reinterpret_cast<float*>(w + W.depth);
    b.rect = reinterpret_cast<int4*>(w + W.rect);
    b.count = reinterpret_cast<uint32_t*>(w + W.count);
    b.offset = reinterpret_cast<uint64_t*>(w + W.offset);
    b.total = reinterpret_cast<unsigned long long*>(w + W.total);
    b.ranges = reinterpret_cast<uint2*>(w + W.ranges);
    b.keys = reinterpret_cast<uint64_t*>(w + W.keys);
    b.keys_alt = reinterpret_cast<uint64_t*>(w + W.keys_alt);
    b.vals = reinterpret_cast<uint32_t*>(w + W.vals);
    b.vals_alt = reinterpret_cast<uint32_t*>(w + W.vals_alt);
    b.scan_temp = w + W.scan;
    b.scan_temp_bytes = W.scan_bytes;
    b.sort_temp = w + W.sort;
    b.sort_temp_bytes = W.sort_bytes;
    b.max_instances = max_instances;
    b.flags = reinterpret_cast<unsigned*>(w);
    hipError_t e = fill_u32(b.flags, 0u, 1, stream);
    if (e == hipSuccess) e = launch_splat_front(n, c, g->means, g->quats, g->log_scales, g->opacity, b, stream);
    if (e != hipSuccess) return hip_status(e, "splat projection");
    unsigned long long total = 0;
    e = hipMemcpyAsync(&total, b.total, sizeof(total), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_status(e, "splat instance count");
    if (instances) *instances = (int64_t)total;
    if ((int64_t)total > max_instances)
        return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "%llu (Gaussian, tile) pairs, workspace holds %lld", total,
                    (long long)max_instances);
    return hip_status(launch_splat_back(n, c, (int64_t)total, colours, colour_stride, b, image, final_T, stream),
                      "splat render");
}

size_t prtgs_glossy_workspace_bytes(const prtgs_transfer_desc* d)
{
    if (!d || d->num_dirs < 1 || d->num_dirs > PRTGS_GLOSSY_MAX_DIRS || (d->sh_bands != 3 && d->sh_bands != 4))
        return 0;
    const size_t S = (size_t)d->num_dirs, K = (size_t)d->sh_bands * d->sh_bands;
    return kFlagBytes + align256(sizeof(float) * 3 * S) + align256(sizeof(float) * K * S);
}

prtgs_status prtgs_glossy_transfer(const prtgs_gaussians* g, const float* roughness, const float* metallic,
                                   const prtgs_transfer_desc* d, const float* vis, float* matrices, void* ws,
                                   size_t ws_bytes, hipStream_t stream)
{
    prtgs_status st = check_gaussians(g, true);
    if (st != PRTGS_OK) return st;
    if (!d) return fail(PRTGS_ERR_INVALID_ARG, "transfer desc is NULL");
    if (d->num_dirs < 1 || d->num_dirs > PRTGS_GLOSSY_MAX_DIRS)
        return fail(PRTGS_ERR_INVALID_ARG, "num_dirs = %d outside [1, %d]", d->num_dirs, PRTGS_GLOSSY_MAX_DIRS);
    if (d->sh_bands != 3 && d->sh_bands != 4)
        return fail(PRTGS_ERR_INVALID_ARG, "glossy matrices take sh_bands 3 or 4 (got %d)", d->sh_bands);
    if (!roughness || !metallic || !vis || !matrices || !ws)
        return fail(PRTGS_ERR_INVALID_ARG, "roughness, metallic, vis, matrices or workspace is NULL");
    if (!aligned256(ws)) return fail(PRTGS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const size_t need = prtgs_glossy_workspace_bytes(d);
    if (ws_bytes < need) return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    const int S = d->num_dirs, K = d->sh_bands * d->sh_bands;
    char* w = static_cast<char*>(ws);
    unsigned* flags = reinterpret_cast<unsigned*>(w);
    float* dirs = reinterpret_cast<float*>(w + kFlagBytes);
    float* Y = reinterpret_cast<float*>(w + kFlagBytes + align256(sizeof(float) * 3 * (size_t)S));
    hipError_t e = fill_u32(flags, 0u, 1, stream);
    if (e == hipSuccess) e = launch_direction_table(S, d->seed, d->sh_bands, nullptr, nullptr, dirs, Y, stream);
    if (e == hipSuccess)
        e = launch_glossy(g->n, S, K, dirs, Y, g->normals, g->albedo, roughness, metallic, vis, matrices, flags,
                          stream);
    return hip_status(e, "glossy transfer");
}

prtgs_status prtgs_glossy_view(int32_t n, int32_t K, const float* matrices, const float* means, const float* eye,
                               float* transfer, hipStream_t stream)
{
    if (n < 0) return fail(PRTGS_ERR_INVALID_ARG, "n < 0");
    if (K != 9 && K != 16) return fail(PRTGS_ERR_INVALID_ARG, "K = %d not 9 or 16", K);
    if (!eye) return fail(PRTGS_ERR_INVALID_ARG, "eye is NULL");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(eye[i])) return fail(PRTGS_ERR_INVALID_ARG, "eye is not finite");
    if (n == 0) return ok();
    if (!matrices || !means || !transfer) return fail(PRTGS_ERR_INVALID_ARG, "matrices, means or transfer is NULL");
    return hip_status(launch_glossy_view(n, K, matrices, means, eye, transfer, stream), "glossy view");
}

prtgs_status prtgs_traversal_stats(const prtgs_gaussians* g, const void* bvh, const prtgs_transfer_desc* d,
                                   int32_t first, int32_t count, uint64_t* stats, void* ws, size_t ws_bytes,
                                   hipStream_t stream)
{
    prtgs_status st = check_desc(d);
    if (st != PRTGS_OK) return st;
    const bool bounce = d->bounces > 0;
    if (bounce && d->bounce_mode != PRTGS_BOUNCE_BLEND)
        return fail(PRTGS_ERR_UNSUPPORTED, "work statistics cover the direct pass and the blended bounce");
    st = check_gaussians(g, bounce);
    if (st != PRTGS_OK) return st;
    const int n = g->n;
    if (!bvh || !ws || !stats) return fail(PRTGS_ERR_INVALID_ARG, "bvh, workspace or stats is NULL");
    if (!aligned256(bvh) || !aligned256(ws)) return fail(PRTGS_ERR_INVALID_ARG, "bvh and workspace must be 256-byte aligned");
    if (first < 0 || count < 0 || (int64_t)first + count > n)
        return fail(PRTGS_ERR_INVALID_ARG, "source range [%d, %d + %d) outside [0, %d)", first, first, count, n);
    if (bounce && (first != 0 || count != n))
        return fail(PRTGS_ERR_INVALID_ARG, "a bounce needs every source's direct transfer: use first = 0, count = n");
    // the counted one-walk blend writes no records: a one-word arena is enough
    prtgs_transfer_desc d1 = *d;
    if (one_walk(d1)) d1.bounce_records = 1;
    d = &d1;
    TransferWs W = transfer_ws_layout(*d, n);
    if (ws_bytes < W.total)
        return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes, W.total);
    char* w = static_cast<char*>(ws);
    hipError_t e = transfer_setup(d, w, W, stream);
    if (e == hipSuccess) e = fill_u32(reinterpret_cast<uint32_t*>(stats), 0u, 16, stream);
    if (e != hipSuccess) return hip_status(e, "traversal stats setup");
    if (count == 0) return ok();
    TransferArgs a = transfer_args(g, bvh, d, first, count, nullptr, nullptr, w, W);
    unsigned long long* st64 = reinterpret_cast<unsigned long long*>(stats);
    if (!bounce) return hip_status(launch_transfer_direct(a, stream, st64), "traversal stats");
    if (one_walk(*d)) return hip_status(launch_fused_stats(a, stream, st64), "traversal stats");
    // the direct pass (its transfers and cut depths feed the walk), then the counted walk
    e = launch_transfer_direct(a, stream);
    if (e == hipSuccess) e = launch_bounce_stats(a, stream, st64);
    return hip_status(e, "traversal stats");
}

prtgs_status prtgs_pack(int64_t count, const float* src, void* dst, prtgs_dtype dtype, hipStream_t stream)
{
    if (count < 0) return fail(PRTGS_ERR_INVALID_ARG, "count < 0");
    if (count == 0) return ok();
    if (!src || !dst) return fail(PRTGS_ERR_INVALID_ARG, "src or dst is NULL");
    if (dtype != PRTGS_BF16 && dtype != PRTGS_F16) return fail(PRTGS_ERR_INVALID_ARG, "pack dtype must be BF16 or F16");
    return hip_status(launch_pack(count, src, dst, dtype, stream), "pack");
}

prtgs_status prtgs_relight(int32_t n, int32_t K, int32_t C, const void* transfer, prtgs_dtype t_dtype, int32_t B,
                           const float* light, void* colour, prtgs_dtype out_dtype, hipStream_t stream)
{
    if (n < 0) return fail(PRTGS_ERR_INVALID_ARG, "n < 0");
    if (K != 1 && K != 4 && K != 9 && K != 16) return fail(PRTGS_ERR_INVALID_ARG, "K = %d not in {1, 4, 9, 16}", K);
    if (C != 1 && C != 3) return fail(PRTGS_ERR_INVALID_ARG, "C = %d not 1 or 3", C);
    if (B < 1 || B > 256) return fail(PRTGS_ERR_INVALID_ARG, "B = %d outside [1, 256]", B);
    if (t_dtype != PRTGS_F32 && t_dtype != PRTGS_BF16 && t_dtype != PRTGS_F16)
        return fail(PRTGS_ERR_INVALID_ARG, "bad transfer dtype");
    if (out_dtype != PRTGS_F32 && out_dtype != PRTGS_F16) return fail(PRTGS_ERR_INVALID_ARG, "colour dtype must be F32 or F16");
    if (n == 0) return ok();
    if (!transfer || !light || !colour) return fail(PRTGS_ERR_INVALID_ARG, "a relight pointer is NULL");
    if ((int64_t)n * B * 3 > ((int64_t)1 << 40)) return fail(PRTGS_ERR_INVALID_ARG, "colour array too large");
    return hip_status(launch_relight(n, K, C, transfer, t_dtype, B, light, colour, out_dtype, stream), "relight");
}

size_t prtgs_relight_backward_workspace_bytes(int32_t n, int32_t K, int32_t C, int32_t B)
{
    if (n < 0 || K < 1 || K > 16 || (C != 1 && C != 3) || B < 1 || B > 256) return 0;
    return relight_backward_ws(n, K, C, B);
}

prtgs_status prtgs_relight_backward(int32_t n, int32_t K, int32_t C, const float* transfer, int32_t B,
                                    const float* light, const float* d_colour, float* d_transfer, float* d_light,
                                    void* ws, size_t ws_bytes, hipStream_t stream)
{
    if (n < 0) return fail(PRTGS_ERR_INVALID_ARG, "n < 0");
    if (K != 1 && K != 4 && K != 9 && K != 16) return fail(PRTGS_ERR_INVALID_ARG, "K = %d not in {1, 4, 9, 16}", K);
    if (C != 1 && C != 3) return fail(PRTGS_ERR_INVALID_ARG, "C = %d not 1 or 3", C);
    if (B < 1 || B > 256) return fail(PRTGS_ERR_INVALID_ARG, "B = %d outside [1, 256]", B);
    if (!d_transfer && !d_light) return ok();
    if (!light || !d_colour || (d_light && !transfer)) return fail(PRTGS_ERR_INVALID_ARG, "a relight pointer is NULL");
    if (!ws || !aligned256(ws)) return fail(PRTGS_ERR_INVALID_ARG, "workspace NULL or not 256-byte aligned");
    size_t need = relight_backward_ws(n, K, C, B);
    if (ws_bytes < need) return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    return hip_status(launch_relight_backward(n, K, C, transfer, B, light, d_colour, d_transfer, d_light, ws, stream),
                      "relight backward");
}

size_t prtgs_transfer_backward_workspace_bytes(const prtgs_transfer_desc* d, int32_t n)
{
    if (!d || n < 1 || check_desc(d) != PRTGS_OK) return 0;
    TransferWs W = transfer_ws_layout(*d, n);
    // + per-leaf scratch gradients: W (9), mu (3), opacity (1), normal (3)
    return W.total + align256(sizeof(float) * 16 * (size_t)n);
}

prtgs_status prtgs_transfer_backward(const prtgs_gaussians* g, const void* bvh, const prtgs_transfer_desc* d,
                                     const float* d_transfer, const float* vis, const prtgs_grads* grads, void* ws,
                                     size_t ws_bytes, hipStream_t stream)
{
    prtgs_status st = check_desc(d);
    if (st != PRTGS_OK) return st;
    if (d->bounces != 0) return fail(PRTGS_ERR_UNSUPPORTED, "the adjoint covers the direct transfer only (bounces = 0)");
    st = check_gaussians(g, false);
    if (st != PRTGS_OK) return st;
    if (!grads) return fail(PRTGS_ERR_INVALID_ARG, "grads struct is NULL");
    if (!bvh || !ws || !d_transfer) return fail(PRTGS_ERR_INVALID_ARG, "bvh, workspace or d_transfer is NULL");
    if (!aligned256(bvh) || !aligned256(ws)) return fail(PRTGS_ERR_INVALID_ARG, "bvh and workspace must be 256-byte aligned");
    const int n = g->n;
    size_t need = prtgs_transfer_backward_workspace_bytes(d, n);
    if (ws_bytes < need) return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    if (!grads->d_means && !grads->d_quats && !grads->d_log_scales && !grads->d_opacity && !grads->d_normals) return ok();

    TransferWs W = transfer_ws_layout(*d, n);
    char* w = static_cast<char*>(ws);
    unsigned* flags = reinterpret_cast<unsigned*>(w);
    float* dirs = reinterpret_cast<float*>(w + W.dirs);
    float* Y = reinterpret_cast<float*>(w + W.Y);
    float* scratch = reinterpret_cast<float*>(w + W.total);
    hipError_t e = fill_u32(flags, 0u, 1, stream);
    if (e == hipSuccess)
        e = launch_direction_table(d->num_dirs, d->seed, d->sh_bands, nullptr, nullptr, dirs, Y, stream);
    if (e == hipSuccess) e = launch_direction_order(d->num_dirs, reinterpret_cast<int32_t*>(w + W.dir_order), stream);
    if (e == hipSuccess) e = fill_u32(reinterpret_cast<uint32_t*>(scratch), 0u, 16 * (size_t)n, stream);
    if (e != hipSuccess) return hip_status(e, "backward setup");

    const BvhLayout L = bvh_layout(n);
    const char* b = static_cast<const char*>(bvh);
    BackwardArgs a{};
    a.fwd.nodes = reinterpret_cast<const Node*>(b + L.nodes);
    a.fwd.prims = reinterpret_cast<const Prim*>(b + L.prims);
    a.fwd.normals = reinterpret_cast<const float4*>(b + L.normals);
    a.fwd.order = reinterpret_cast<const int32_t*>(b + L.order);
    a.fwd.dirs = dirs;
    a.fwd.Y = Y;
    a.fwd.dir_order = reinterpret_cast<const int32_t*>(w + W.dir_order);
    a.fwd.S = d->num_dirs;
    a.fwd.K = d->sh_bands * d->sh_bands;
    a.fwd.n = n;
    a.fwd.first = 0;
    a.fwd.count = n;
    a.fwd.channels = 1;
    a.fwd.hp = hit_params(*d);
    a.fwd.transfer = nullptr;
    a.fwd.vis = nullptr;
    a.fwd.hit_table = nullptr;
    a.fwd.albedo = nullptr;
    a.fwd.G = group_size(n, d->sources_per_wave);
    a.fwd.Q_req = d->direction_parts;
    a.fwd.flags = flags;
    a.d_transfer = d_transfer;
    a.vis_in = vis;
    a.g_W = scratch;
    a.g_mu = scratch + 9 * (size_t)n;
    a.g_o = scratch + 12 * (size_t)n;
    a.g_n = scratch + 13 * (size_t)n;
    a.quats = g->quats;
    a.log_scales = g->log_scales;
    a.out = *grads;
    return hip_status(launch_transfer_backward(a, stream), "transfer backward");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The direct transfer without a caller workspace.  Its scratch (flag word,
// direction tables, per-ray weights) is this file's static device array;
// each GPU holds its own copy, whose address hipGetSymbolAddress gives once
// per device (the name itself is only a host-side stand-in).
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)PRTGS_NOALLOC_SCRATCH_MIB << 20;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// The current device's copy of `scratch` (looked up on its first use).
hipError_t scratch_on_current_device(char** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u)) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<char*>(g_scratch_ptr[dev]);
    return hipSuccess;
}

}  // namespace

extern "C" {

prtgs_status prtgs_precompute_transfer_noalloc(const prtgs_gaussians* g, const void* bvh, const prtgs_transfer_desc* d,
                                               int32_t first, int32_t count, float* transfer, float* vis,
                                               unsigned* flags, hipStream_t stream)
{
    prtgs_status st = check_desc(d);
    if (st != PRTGS_OK) return st;
    if (d->bounces != 0)
        return fail(PRTGS_ERR_UNSUPPORTED, "the no-allocation transfer covers the direct pass only (bounces = 0)");
    st = check_gaussians(g, false);
    if (st != PRTGS_OK) return st;
    const int n = g->n;
    if (!bvh) return fail(PRTGS_ERR_INVALID_ARG, "bvh is NULL");
    if (!aligned256(bvh)) return fail(PRTGS_ERR_INVALID_ARG, "bvh must be 256-byte aligned");
    if (first < 0 || count < 0 || (int64_t)first + count > n)
        return fail(PRTGS_ERR_INVALID_ARG, "source range [%d, %d + %d) outside [0, %d)", first, first, count, n);
    if (count > 0 && !transfer) return fail(PRTGS_ERR_INVALID_ARG, "transfer is NULL");
    // per-ray weights are held for the selected sources only: lay the
    // scratch out as a workspace for `count` sources
    TransferWs W = transfer_ws_layout(*d, count > 0 ? count : 1);
    if (W.total > kNoAllocScratchBytes)
        return fail(PRTGS_ERR_WORKSPACE_TOO_SMALL,
                    "%d sources x %d directions need %zu bytes of scratch, the library holds %zu: use fewer sources per "
                    "call",
                    count, d->num_dirs, W.total, kNoAllocScratchBytes);
    char* w = nullptr;
    hipError_t e = scratch_on_current_device(&w);
    if (e != hipSuccess) return hip_status(e, "scratch address");
    unsigned* fl = flags ? flags : reinterpret_cast<unsigned*>(w);
    e = fill_u32(fl, 0u, 1, stream);
    if (e == hipSuccess)
        e = launch_direction_table(d->num_dirs, d->seed, d->sh_bands, nullptr, nullptr,
                                   reinterpret_cast<float*>(w + W.dirs), reinterpret_cast<float*>(w + W.Y), stream);
    if (e == hipSuccess) e = launch_direction_order(d->num_dirs, reinterpret_cast<int32_t*>(w + W.dir_order), stream);
    if (e != hipSuccess) return hip_status(e, "direction table");
    if (count == 0) return ok();
    TransferArgs a = transfer_args(g, bvh, d, first, count, transfer, vis, w, W);
    a.flags = fl;
    return hip_status(launch_transfer_direct(a, stream), "direct transfer");
}

}  // extern "C"
