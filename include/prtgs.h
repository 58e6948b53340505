/*
 * prtgs.h -- C ABI of the MI355X (gfx950) radiance-transfer library for 3D
 * Gaussian splats (PRTGS, arXiv 2408.03538).
 *
 * The library precomputes, for every splat, the diffuse radiance transfer
 * vector of Sec. 3.2 / Sec. 4.5: the visibility along S directions, traced
 * from the splat centre through the other 3D Gaussians (Sec. 4.4), times
 * max(0, n . w), projected onto real spherical harmonics (Eq. 7, 9, 11, 29);
 * optionally one interreflection bounce (Eq. 20-22, 30-33); relights splats
 * under many SH light environments with the dot product of Eq. 14; and runs
 * the adjoint of both.
 *
 * Conventions shared by every entry point:
 *  - Every array pointer is a DEVICE pointer unless the comment says "host".
 *    Arrays are dense, row-major, 32-bit float unless stated.
 *  - The caller owns every buffer.  The library allocates no device memory:
 *    BVH storage and scratch ("workspace") are caller buffers whose sizes come
 *    from the *_bytes queries.  Workspaces must be 256-byte aligned.
 *  - Every call only enqueues work on `stream` and returns.  Arguments are
 *    validated on the host first; on any error nothing is enqueued and the
 *    status says why (prtgs_last_error() gives a message, per thread).
 *  - Device-side conditions (non-finite inputs, traversal stack overflow) set
 *    bits in the 32-bit flag word at byte 0 of the call's workspace.  The
 *    word is cleared by the call; read it after synchronising the stream.
 *  - Calls on distinct buffers may run concurrently.
 */
#ifndef PRTGS_H
#define PRTGS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PRTGS_ABI_VERSION 5   /* 5: one-walk blended bounce (bounce_records in prtgs_transfer_desc) */

typedef enum {
    PRTGS_OK = 0,
    PRTGS_ERR_INVALID_ARG = 1,        /* bad size, null pointer, out-of-range parameter */
    PRTGS_ERR_WORKSPACE_TOO_SMALL = 2,/* a caller buffer is smaller than its *_bytes query */
    PRTGS_ERR_UNSUPPORTED = 3,        /* valid request this version does not implement */
    PRTGS_ERR_HIP = 4                 /* a HIP runtime call or kernel launch failed */
} prtgs_status;

typedef enum { PRTGS_F32 = 0, PRTGS_BF16 = 1, PRTGS_F16 = 2 } prtgs_dtype;

/* Device flag bits (flag word at byte 0 of a workspace). */
#define PRTGS_FLAG_NONFINITE 0x1u       /* a non-finite value reached a kernel */
#define PRTGS_FLAG_STACK_OVERFLOW 0x2u  /* BVH deeper than the traversal stack */
#define PRTGS_FLAG_BAD_TREE 0x4u        /* malformed BVH (wrong buffer or n): traversal stopped */
#define PRTGS_FLAG_BAD_INDEX 0x8u       /* an index-matrix entry outside [-1, n): skipped */
#define PRTGS_FLAG_RECORDS_DEFERRED 0x20u /* not an error: the one-walk blended bounce ran out of
                                           record space and redid part of the work with two walks */
#define PRTGS_FLAG_ROUND_CAP 0x10u      /* a bounce ray needed more than PRTGS_BOUNCE_MAX_ROUNDS
                                           traversals; its walk stopped there */

/* The splats (Sec. 3.1, Eq. 1-2; normal Sec. 4.3; albedo Sec. 4.2).
 * Caller-owned, read-only during calls. */
typedef struct {
    int32_t n;                 /* number of Gaussians, >= 1 */
    const float* means;        /* [n][3] centres */
    const float* quats;        /* [n][4] rotation (w, x, y, z); normalised inside */
    const float* log_scales;   /* [n][3] log of the scales S of Eq. 2 */
    const float* opacity;      /* [n]    learned opacity, in (0, 1] */
    const float* normals;      /* [n][3] unit normals */
    const float* albedo;       /* [n][3] diffuse albedo rho; needed only for bounces >= 1 */
} prtgs_gaussians;

/* Parameters of the transfer (Sec. 4.4-4.5).  The cutoffs are the reading of
 * the paper used throughout: a Gaussian is hit by a ray iff its peak density
 * along the ray lies at t* > t_min and there d^2 <= sigma_cut^2; then
 * alpha = min(opacity exp(-d^2/2), alpha_max) (Eq. 27 as read here), ignored
 * if below alpha_min; transmittance below T_eps counts as fully occluded. */
typedef struct {
    int32_t num_dirs;          /* S directions per splat, 1 .. 65536 */
    int32_t sh_bands;          /* L bands, K = L*L coefficients; 1 .. 4 */
    uint64_t seed;             /* seed of the stratified direction jitter */
    int32_t bounces;           /* interreflection bounces: 0 (direct transfer only), 1 with
                                  PRTGS_BOUNCE_BLEND, 0 .. 8 with PRTGS_BOUNCE_INDEX */
    float sigma_cut;           /* 3.0 */
    float t_min;               /* 0.0 */
    float T_eps;               /* 1e-4 */
    float alpha_min;           /* 0.0 */
    float alpha_max;           /* 0.99 */
    int32_t bounce_mode;       /* PRTGS_BOUNCE_BLEND or PRTGS_BOUNCE_INDEX */
    float t_same;              /* index mode: hits with transmittance in front above it are not
                                  candidates (same-surface filter); (0, 1], 1 = off */
    /* Work split (0 = chosen by the library from the number of sources).  It
     * changes only the order in which each ray's factors (1 - alpha) are
     * multiplied and, for the blended bounce, how the per-direction sums are
     * grouped before they are added: the last bits of the result. */
    int32_t sources_per_wave;  /* sources traced together by one wave: 1 (one source per wave, its
                                  hemisphere directions compacted), 2, 4, 8, 16, 32 or 64 */
    int32_t direction_parts;   /* waves that share one source group's directions, 1 .. 64; the
                                  blended bounce keeps at most PRTGS_BLEND_PARTS_MAX of them */
    /* Blended bounce (bounces == 1, PRTGS_BOUNCE_BLEND) in one walk per ray
     * instead of two: the walk that blends a ray's hits also yields its
     * visibility, so no separate direct pass runs; the blended hits' weights
     * (8 bytes each, about 38 per traced ray of a million-splat scene) wait in
     * a record arena of this many 8-byte words in the workspace until every
     * direct transfer exists.  Work whose records do not fit is redone by the
     * two-walk method (PRTGS_FLAG_RECORDS_DEFERRED); the results agree with the
     * two-walk method to the last bits of the visibility products.  0 = two
     * walks (no arena).  With PRTGS_BOUNCE_INDEX any value > 0 makes the walk
     * that builds the index matrix give the visibility too (no direct pass, no
     * arena: it keeps only each ray's chosen hit). */
    int64_t bounce_records;
} prtgs_transfer_desc;

#define PRTGS_BLEND_PARTS_MAX 64    /* blended bounce: direction parts with sums of their own */
#define PRTGS_BOUNCE_HIT_LIST 256   /* bounce walk: hits a ray lists per traversal round */
#define PRTGS_BOUNCE_MAX_ROUNDS 4096 /* bounce walk: traversal rounds per ray (each blends >= 1 hit) */

/* How a bounce weighs the hits of a ray.
 * BLEND: every hit front to back with weight alpha_j T_j (depth-ordered alpha
 *   blend), one bounce.
 * INDEX: the paper's own scheme (Sec. 4.4 Eq. 26, Sec. 4.5 Eq. 32-35): per ray
 *   only the hit of largest W_j = alpha_j T_j max(-w . n_j, 0) among hits with
 *   T_j <= t_same (an index matrix, -1 = none), with full weight; bounce m
 *   gathers bounce m - 1 of the indexed splats, no re-tracing. */
enum { PRTGS_BOUNCE_BLEND = 0, PRTGS_BOUNCE_INDEX = 1 };
#define PRTGS_MAX_INDEX_BOUNCES 8

/* Gradients (each pointer may be NULL = not wanted).  Accumulated (+=) into
 * caller-initialised buffers of the shapes of prtgs_gaussians. */
typedef struct {
    float* d_means;            /* [n][3] */
    float* d_quats;            /* [n][4] with respect to the unnormalised quaternion */
    float* d_log_scales;       /* [n][3] */
    float* d_opacity;          /* [n] */
    float* d_normals;          /* [n][3] */
} prtgs_grads;

int32_t prtgs_abi_version(void);
const char* prtgs_last_error(void);            /* host string, thread-local, never NULL */
const char* prtgs_status_string(prtgs_status s);

/* ---------------------------------------------------------------------- */
/* Direction table (Eq. 8-11 need the SH basis at a set of directions).     */
/* S stratified equal-area directions: grid n_u x n_v with n_u the largest  */
/* divisor of S not above floor(sqrt(S)); stratum s = a n_v + b gets        */
/* z = 1 - 2 (a + xi)/n_u, phi = 2 pi (b + eta)/n_v with xi, eta the top 53 */
/* bits (scaled by 2^-53) of outputs 2s and 2s+1 of a SplitMix64 stream     */
/* seeded with `seed`.  Generated in FP64 on the device, rounded to FP32;   */
/* Y is the real orthonormal SH basis (Condon-Shortley phase, index         */
/* k = l^2 + l + m) at the normalised FP32 direction, in FP64.              */
/* Any output pointer may be NULL.  Quadrature weight of each: 4 pi / S.    */
/* ---------------------------------------------------------------------- */
prtgs_status prtgs_direction_table(int32_t num_dirs, uint64_t seed, int32_t sh_bands,
                                   double* dirs64 /* [S][3] */, double* Y64 /* [S][K] */,
                                   float* dirs32 /* [S][3] */, float* Y32 /* [S][K] */,
                                   hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Bounding volume hierarchy over the Gaussians' 3-sigma boxes (the paper   */
/* builds its Gaussian ray tracer on a BVH, Sec. 4.4).  Linear BVH: 30-bit  */
/* Morton codes of the centres, a stable radix sort, Karras' hierarchy      */
/* (ties broken by index) and a bottom-up box refit.  The BVH buffer also   */
/* holds per-splat ray-test records (centre, opacity, whitening matrix      */
/* diag(1/s) R^T, normal) in leaf order and the leaf-to-splat permutation.   */
/* The BVH depends on means, quats, log_scales, opacity, normals; rebuild   */
/* it when any of them changes.  ws: scratch of prtgs_build_workspace_bytes.*/
/* ---------------------------------------------------------------------- */
size_t prtgs_bvh_bytes(int32_t n);
size_t prtgs_build_workspace_bytes(int32_t n);
prtgs_status prtgs_build_bvh(const prtgs_gaussians* g /* host struct */, void* bvh, size_t bvh_bytes,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/* Leaf order of a built BVH: order[r] = index of the Gaussian in leaf r (a
 * copy into caller memory, enqueued on stream). */
prtgs_status prtgs_bvh_leaf_order(const void* bvh, int32_t n, int32_t* order /* [n] */,
                                  hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Transfer precompute (Sec. 4.4-4.5; Eq. 7, 9, 29; bounce Eq. 20-22, 30-33).*/
/* For each source i and direction w_s with c = n_i . w_s > 0 the ray       */
/* mu_i + t w_s is traced through every Gaussian j != i; V = prod (1 -      */
/* alpha_j) over hits (0 if below T_eps);                                   */
/*   t_dir[i][k] = (4 pi / S) sum_s V c Y_k(w_s).                           */
/* The stored transfer excludes the receiver's rho_i / pi (multiply the     */
/* relit value by it).  With bounces == 1 the hits of each ray are also     */
/* walked front to back (by t*, then leaf order), hit j getting weight      */
/* alpha_j T_j with T_j the transmittance in front of it, until the         */
/* transmittance drops below T_eps, and                                     */
/*   transfer[i][c][:] = t_dir[i][:] + (4 pi/S) sum_s c sum_j w_j rho_jc/pi t_dir[j][:].*/
/* With bounce_mode PRTGS_BOUNCE_INDEX the bounces follow the index matrix  */
/* (see prtgs_index_matrix, prtgs_self_transfer):                           */
/*   transfer[i][c][:] = t_dir[i][:] + sum_{m=1..bounces} T^m[i][c][:].     */
/* transfer: [n][C][K], C = 1 (bounces 0) or 3 (bounces >= 1), written for the */
/* selected sources only.  Sources are selected by leaf rank: those in     */
/* leaf positions [first, first + count) (chunked or resumable runs; with  */
/* bounces == 1 the range must be the whole scene).  vis (may be NULL):     */
/* [n][S] visibility of every ray of the selected sources, -1 for rays with */
/* c <= 0 (not traced).  ws: prtgs_transfer_workspace_bytes: 4 n S bytes  */
/* of per-ray weights (2 GiB at 1M x 512); with a bounce also 4 n S bytes   */
/* of per-ray cut depths and the per-lane hit lists of the persistent      */
/* waves: min(n, 4096) waves and 768 MiB of lists + 512 MiB of hit records */
/* (with bounce_records > 0: min(n, 7168) waves, 1344 + 896 MiB)           */
/* + 12 K Q n bytes of bounce sums for the blend (Q = the direction parts  */
/* it keeps: 64 by default from 16 sources per wave at S >= 256, 12.3 GB  */
/* at 1M x 512; fewer parts, fewer bytes), min(n, 5120) waves and 960 MiB */
/* of lists in index mode.  With bounce_records > 0 also the record arena  */
/* (8 bounce_records bytes) and 12 bytes per work item (Q per source group). */
/* ---------------------------------------------------------------------- */
size_t prtgs_transfer_workspace_bytes(const prtgs_transfer_desc* d /* host */, int32_t n);
prtgs_status prtgs_precompute_transfer(const prtgs_gaussians* g /* host */, const void* bvh,
                                       const prtgs_transfer_desc* d /* host */, int32_t first,
                                       int32_t count, float* transfer, float* vis, void* ws,
                                       size_t ws_bytes, hipStream_t stream);

/* The direct transfer (bounces == 0) as prtgs_precompute_transfer computes  */
/* it, for callers that cannot allocate (code under HIP graph capture, tight  */
/* serving loops, harnesses that forbid allocation): no workspace argument;  */
/* its scratch (flag word, direction tables, 4 count S bytes of per-ray      */
/* weights) is a static device array of PRTGS_NOALLOC_SCRATCH_MIB MiB inside */
/* the library, one per GPU it runs on, held until the process ends.  The    */
/* call makes no allocation.  Call it with the device of `stream` current.   */
/* count x S beyond the scratch (about 16.7M rays, e.g. 32,000 sources at    */
/* S = 512) returns PRTGS_ERR_WORKSPACE_TOO_SMALL with nothing enqueued:     */
/* cover larger scenes with several source ranges.  Calls that overlap on    */
/* one GPU share its scratch and race: serialise them (one stream, or        */
/* events).  bounces != 0 returns PRTGS_ERR_UNSUPPORTED.  flags (device word,*/
/* may be NULL): cleared, then receives the call's device flag bits; with    */
/* NULL they go to the scratch's own flag word and are not reported.  The    */
/* result equals prtgs_precompute_transfer's for the same arguments.         */
#define PRTGS_NOALLOC_SCRATCH_MIB 64
prtgs_status prtgs_precompute_transfer_noalloc(const prtgs_gaussians* g /* host */, const void* bvh,
                                               const prtgs_transfer_desc* d /* host */, int32_t first,
                                               int32_t count, float* transfer, float* vis, unsigned* flags,
                                               hipStream_t stream);

/* Index matrix of the paper's bounce (Sec. 4.4, Eq. 26 and the same-surface */
/* filter): index[i][s] = the Gaussian (original index) of largest           */
/* W_j = alpha_j T_j max(-w_s . n_j, 0) along the ray of source i in          */
/* direction s among the hits with T_j <= d->t_same, hits walked in (t*,     */
/* leaf rank) order up to the one that takes the transmittance below T_eps   */
/* (the nearer one on equal weights); -1 if no hit has W > 0 or c <= 0.      */
/* Traces the direct pass first (its depths bound the walk).  index: [n][S] */
/* int32, every source.  ws: prtgs_transfer_workspace_bytes of d with        */
/* bounce_mode = PRTGS_BOUNCE_INDEX and bounces >= 1.                        */
prtgs_status prtgs_index_matrix(const prtgs_gaussians* g /* host */, const void* bvh,
                                const prtgs_transfer_desc* d /* host */, int32_t* index, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* One step of the paper's recursive self-transfer (Sec. 4.5 Eq. 32-34):     */
/*   t_out[i][c][k] = (4 pi / S) sum_{s: index[i][s] >= 0, c_is > 0}          */
/*                    c_is (albedo[j][c] / pi) t_prev[j][c'][k],              */
/* j = index[i][s], c_is = normals[i] . dirs[s], c' = c if c_prev == 3 else  */
/* 0.  dirs: [S][3] FP32 (prtgs_direction_table); normals, albedo [n][3];    */
/* index [n][S]; t_prev [n][c_prev][K]; t_out [n][3][K] (overwritten; must  */
/* not alias t_prev).  Index entries outside [-1, n) are skipped and set    */
/* PRTGS_FLAG_BAD_INDEX in *flags (a device word; may be NULL).              */
prtgs_status prtgs_self_transfer(int32_t n, int32_t S, int32_t K, const float* dirs, const float* normals,
                                 const float* albedo, const int32_t* index, const float* t_prev,
                                 int32_t c_prev, float* t_out, unsigned* flags, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Gaussian splatting of per-splat colours (the rasterizer the paper renders*/
/* with, Sec. 3.1: Sigma = R S S^T R^T, footprint Sigma' = J W Sigma W^T J^T,*/
/* front-to-back blending of Eq. 4), e.g. of prtgs_relight's colours.  With */
/* x_c = view * [x; 1] (camera looks along +z), a Gaussian with x_c.z >=     */
/* near_z projects to u = fx x/z + cx, v = fy y/z + cy with the 2D          */
/* covariance J M diag(s^2) M^T J^T + 0.3 I (J the projection's Jacobian    */
/* with x/z, y/z held within 1.3 x the frustum, M = view rotation x R(q)).   */
/* Pixel (px, py) at (px + 0.5, py + 0.5) takes, in increasing camera depth */
/* (then index), every Gaussian with alpha = min(0.99, o exp(-d^T Sigma'^-1 */
/* d / 2)) >= 1/255, C += c alpha T, T *= 1 - alpha, and stops before the   */
/* Gaussian that would take T below 1e-4; image = C + T background.          */
typedef struct {
    float view[12];            /* world-to-camera [R | t], row-major 3 x 4 */
    float fx, fy, cx, cy;      /* intrinsics, pixels */
    int32_t width, height;     /* image size, pixels (1 .. 16384) */
    float near_z;              /* Gaussians nearer than this are culled (> 0) */
    float background[3];
} prtgs_camera;

/* Workspace for n Gaussians and up to max_instances (Gaussian, tile) pairs. */
size_t prtgs_splat_workspace_bytes(int32_t n, int32_t width, int32_t height, int64_t max_instances);
/* colours: [n] RGB rows with colour_stride floats between rows (3 for an   */
/* [n][3] array; 3B to pick one light of prtgs_relight's [n][B][3]).  image:*/
/* [height][width][3] FP32; final_T: [height][width] or NULL.  Synchronises  */
/* `stream` once, to read the number of (Gaussian, tile) pairs (returned in */
/* *instances, host, may be NULL); more than max_instances (or 2^32) fails  */
/* with PRTGS_ERR_WORKSPACE_TOO_SMALL and renders nothing.  Non-finite      */
/* Gaussians set PRTGS_FLAG_NONFINITE and are skipped.                      */
prtgs_status prtgs_splat_render(const prtgs_gaussians* g /* host */, const float* colours, int64_t colour_stride,
                                const prtgs_camera* cam /* host */, float* image, float* final_T,
                                int64_t max_instances, void* ws, size_t ws_bytes, int64_t* instances /* host */,
                                hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Glossy transfer matrices (Sec. 4.5, Eq. 36-41) with the BRDF of Sec. 4.2: */
/*   f(wi, wo) = (1 - m) rho / pi + D F G / (4 (wi . n)(wo . n)),           */
/* D = GGX with alpha = r^2, F = Schlick with F0 = 0.04 (1 - m) + m rho,     */
/* G = Smith with Schlick-GGX G1(x) = x / (x (1 - k) + k), k = (r + 1)^2 / 8 */
/* (the paper leaves D, F, G to a supplement; these are the usual choices), */
/* and with T(wi, wo) = f (wi . n) V(wi):                                     */
/*   matrices[i][c][a][b] = (4 pi / S)^2 sum_s sum_p Y_a(w_s) T_c(w_s, w_p)  */
/*                          Y_b(w_p)                                          */
/* over the S stratified directions of d (seed, num_dirs <= 512, sh_bands 3  */
/* or 4) as both input (s) and output (p) directions, T = 0 outside the     */
/* upper hemisphere of the (normalised) normal.  The outgoing radiance of   */
/* splat i seen from wo under light l is sum_b (sum_a l_a M[a][b]) Y_b(wo).  */
/* roughness [n] in (0, 1], metallic [n] in [0, 1], albedo from g; vis:     */
/* [n][S] per-ray visibility as written by prtgs_precompute_transfer (read  */
/* where n . w > 0; negative entries count as 0).  matrices: [n][3][K][K]   */
/* FP32, overwritten.  A splat with a zero or non-finite normal or material  */
/* outside range gets zeros and sets PRTGS_FLAG_NONFINITE.                   */
#define PRTGS_GLOSSY_MAX_DIRS 512
size_t prtgs_glossy_workspace_bytes(const prtgs_transfer_desc* d /* host */);
prtgs_status prtgs_glossy_transfer(const prtgs_gaussians* g /* host */, const float* roughness,
                                   const float* metallic, const prtgs_transfer_desc* d /* host */,
                                   const float* vis, float* matrices, void* ws, size_t ws_bytes,
                                   hipStream_t stream);
/* The per-frame view step: transfer[i][c][a] = sum_b matrices[i][c][a][b]  */
/* Y_b(w_i), w_i = (eye - means[i]) / |eye - means[i]| (the basis in FP64),  */
/* a transfer vector [n][3][K] that prtgs_relight turns into colours.       */
/* eye: host float[3].  A splat at the eye gets zeros.                       */
prtgs_status prtgs_glossy_view(int32_t n, int32_t K, const float* matrices, const float* means,
                               const float* eye /* host */, float* transfer, hipStream_t stream);

/* Work statistics (nothing else is written).  Direct pass (bounces == 0),
 * over the selected sources: stats[0] traced rays, stats[1] child-box tests
 * and stats[2] Gaussian tests that a single-ray depth-first traversal of this
 * BVH (same child order, same early termination) performs, summed over rays;
 * stats[3] node visits and stats[4] Gaussian-record visits of the wave
 * packets, summed.  Blended bounce (bounces == 1, PRTGS_BOUNCE_BLEND; every
 * source): the direct pass runs, then the bounce walk is counted the same way
 * (stats[0] its traced rays, [1]-[4] its traversal work over every round and
 * the depth intervals it walks), with stats[5] the hits blended (those with
 * transmittance >= T_eps in front: the contributing hits), stats[6] the hits
 * listed and stats[7] the traversal rounds, each summed over rays; with
 * bounce_records > 0 the one walk that replaces both is counted (stats[0] its
 * traced rays, the rest as for the bounce walk).  stats: device array of 8
 * uint64, overwritten.  ws as for prtgs_precompute_transfer with the same d,
 * except that no record arena is needed (the size for bounce_records = 1).
 * Index mode: PRTGS_ERR_UNSUPPORTED. */
prtgs_status prtgs_traversal_stats(const prtgs_gaussians* g /* host */, const void* bvh,
                                   const prtgs_transfer_desc* d /* host */, int32_t first, int32_t count,
                                   uint64_t* stats, void* ws, size_t ws_bytes, hipStream_t stream);

/* Round a float32 array to bf16 or f16 storage (round to nearest even),
 * e.g. transfer vectors before relighting.  dst has `count` 2-byte values. */
prtgs_status prtgs_pack(int64_t count, const float* src, void* dst, prtgs_dtype dtype,
                        hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Relighting (Eq. 14, Eq. 41 for a vector transfer): per splat and light   */
/* environment the outgoing value is the dot product of transfer and light  */
/* SH,  colour[i][b][c] = sum_k transfer[i][c'][k] light[b][c][k],  with    */
/* c' = c if C == 3 else 0.  transfer [n][C][K] in t_dtype (F32, BF16, F16);*/
/* light [B][3][K] F32; colour [n][B][3] in out_dtype (F32 or F16).  The    */
/* 16-bit path runs on MFMA with FP32 accumulation and the light split into */
/* a high and a low bf16/f16 part, so its error is set by the storage of     */
/* transfer and colour.  F32 transfer and colour with K = 4 or 16 and at     */
/* least 16 lights run on FP32 MFMA (the same FP32 products, summed in       */
/* another order than the one-thread-per-colour form used otherwise).        */
/* K in {1, 4, 9, 16}, C in {1, 3}, 1 <= B <= 256.                           */
/* ---------------------------------------------------------------------- */
prtgs_status prtgs_relight(int32_t n, int32_t K, int32_t C, const void* transfer, prtgs_dtype t_dtype,
                           int32_t B, const float* light, void* colour, prtgs_dtype out_dtype,
                           hipStream_t stream);

/* Adjoint of prtgs_relight for F32 transfer and colour (both outputs are
 * overwritten, not accumulated):
 *   d_transfer[i][c'][k] = sum_b sum_{c mapped to c'} d_colour[i][b][c] light[b][c][k]
 *   d_light[b][c][k]     = sum_i d_colour[i][b][c] transfer[i][c'][k]  (compensated sums)
 * Either output may be NULL.  ws: prtgs_relight_backward_workspace_bytes. */
size_t prtgs_relight_backward_workspace_bytes(int32_t n, int32_t K, int32_t C, int32_t B);
prtgs_status prtgs_relight_backward(int32_t n, int32_t K, int32_t C, const float* transfer, int32_t B,
                                    const float* light, const float* d_colour, float* d_transfer,
                                    float* d_light, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Adjoint of the direct transfer (bounces == 0): given d_transfer [n][1][K]*/
/* = dLoss/dt_dir, accumulates dLoss/d(means, quats, log_scales, opacity,   */
/* normals) into `grads`.  Hit lists are not stored: every ray is traced    */
/* again for its per-hit terms.  vis (may be NULL): the [n][S] visibilities */
/* that prtgs_precompute_transfer returned for the same Gaussians, BVH and  */
/* parameters over all sources; with it each ray is traced once, without it */
/* twice (visibility first).  The gradient is that of the piecewise-smooth  */
/* forward with the hit, hemisphere and opacity-cutoff decisions held       */
/* fixed.  Atomic accumulation: summation order, hence the last bits, may   */
/* vary between runs.  ws: prtgs_transfer_backward_workspace_bytes.         */
/* ---------------------------------------------------------------------- */
size_t prtgs_transfer_backward_workspace_bytes(const prtgs_transfer_desc* d /* host */, int32_t n);
prtgs_status prtgs_transfer_backward(const prtgs_gaussians* g /* host */, const void* bvh,
                                     const prtgs_transfer_desc* d /* host */, const float* d_transfer,
                                     const float* vis, const prtgs_grads* grads /* host struct */,
                                     void* ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PRTGS_H */
