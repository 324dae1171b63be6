/*
 * lsdf.h -- C ABI of liblsdf.so: batched robot-to-obstacle clearance against
 * link-local signed distance grids on AMD Instinct MI355X (gfx950).
 *
 * The method (Fujii & Pham, "Real-time Batched Distance Computation for
 * Time-Optimal Safe Path Tracking", Sec. III-A): for every configuration
 * theta_c of a D-DoF arm, forward kinematics gives the pose T_{i,c} of every
 * link i; the distance between the robot and the obstacles at theta_c is the
 * minimum, over the occupied obstacle voxels x_j and the links i, of link
 * i's precomputed signed distance field ("Link SDF") read at the obstacle
 * expressed in the link's frame.  This library evaluates that minimum
 * directly per point (each point is moved into every link frame by the
 * inverse pose of Sec. III-B-1, Eq. 4, and the link grid is sampled by
 * trilinear interpolation), rather than through the paper's pre-aligned
 * per-configuration robot grids.
 *
 * Conventions shared by every call
 *   - Return value: LSDF_OK (0) or a negative LSDF_E_* code.  No exception
 *     crosses the ABI.  lsdf_last_error() gives a message for the last
 *     failure on the calling thread.
 *   - Argument errors are detected on the host before anything is enqueued;
 *     on error nothing is launched and no output is touched.
 *   - Device pointers refer to memory of the current HIP device.  All work
 *     is enqueued asynchronously on `stream` (a hipStream_t passed as void*;
 *     NULL = the legacy default stream).  Device faults surface at the
 *     caller's next synchronisation.
 *   - The library never allocates memory.  All buffers are owned by the
 *     caller; scratch memory comes from a caller-provided workspace.
 *   - Inputs must be finite.  Units are metres and radians.
 *   - Poses are row-major 3x4 [R | t] mapping link-frame coordinates to world
 *     coordinates: x_world = R x_link + t.
 */
#ifndef LSDF_H
#define LSDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define LSDF_OK             0
#define LSDF_E_INVALID_ARG (-1)   /* NULL pointer, non-finite or out-of-range value */
#define LSDF_E_SHAPE       (-2)   /* inconsistent sizes, workspace too small */
#define LSDF_E_UNSUPPORTED (-3)   /* unknown dtype or flag */
#define LSDF_E_DEVICE      (-4)   /* a HIP call failed (launch error, bad stream) */

/* ---- grid storage types -------------------------------------------------- */
#define LSDF_F32  0
#define LSDF_BF16 1
#define LSDF_F16  2

/* ---- limits --------------------------------------------------------------- */
#define LSDF_MAX_LINKS      16    /* links per query (dof + 1 for a serial arm) */
#define LSDF_MAX_DOF        15
#define LSDF_MAX_COMPONENTS 16    /* closed parts per link mesh */
#define LSDF_MAX_TRAJECTORIES 65536          /* trajectories per batched query */
#define LSDF_FRNN_HIDDEN      32             /* hidden units of the grid-transformation network */
#define LSDF_FRNN_MAX_HALF    64             /* its largest block half-width m (voxels) */
#define LSDF_MAX_POINTS (((int64_t)1) << 34) /* obstacle points per query */

/* One link's SDF grid (the "Link SDF" of Sec. III-A: extent e_r, resolution
 * r_r, in the link's own frame).  Node-centred: node k = (kx, ky, kz),
 * 0 <= k_a < n_a, holds the signed distance at lo + k * h with
 * h_a = (hi_a - lo_a) / (n_a - 1); the box [lo, hi] is the capture range.
 * Storage: element (kz * n_y + ky) * n_x + kx (x fastest), `dtype` elements,
 * starting `elem_offset` elements into the shared grid buffer.  Negative
 * inside the link, positive outside.  16-bit storage (bfloat16 or IEEE
 * binary16) is widened exactly to FP32 before interpolation; interpolation
 * and every reduction stay FP32.  The grids of one query share a dtype. */
typedef struct lsdf_grid {
    float   lo[3];
    float   hi[3];
    int32_t n[3];          /* nodes per axis, each >= 2 */
    int32_t dtype;         /* storage: LSDF_F32, LSDF_BF16 or LSDF_F16 */
    int64_t elem_offset;   /* >= 0, in elements of `dtype` */
} lsdf_grid;

/* One joint of a standard (distal) Denavit-Hartenberg chain: frame k is
 * frame k-1 moved by Rz(q_k + theta_offset) Tz(d) Tx(a) Rx(alpha). */
typedef struct lsdf_dh {
    float a;
    float alpha;
    float d;
    float theta_offset;
} lsdf_dh;

/* Library version, (major << 16) | (minor << 8) | patch. */
int lsdf_version(void);

/* Message describing the last failed call on this thread ("" if none).  The
 * pointer stays valid until the next library call on the same thread. */
const char* lsdf_last_error(void);

/* Measurement aid: the calling thread's next clearance query (plain,
 * batched or learned) records `before` on its stream just before launching
 * its main kernel and `after` just after it, so that the elapsed time
 * between the two events is that kernel's alone (without the small set-up
 * and finalising kernels around it).  before and after are hipEvent_t
 * created by the caller, passed as void*; both or neither (NULL, NULL
 * clears the setting).  The setting is used by one query and then cleared;
 * a query whose point count is 0 launches no main kernel and leaves it. */
int lsdf_set_kernel_events(void* before, void* after);

/* ---- forward kinematics ----------------------------------------------------
 * Sec. III-A: the transformations T_{i,c} of every link i at every
 * configuration c, by forward kinematics run in parallel over c.
 *   dh      host [dof] joint parameters, 1 <= dof <= LSDF_MAX_DOF
 *   base_T  host [3][4] pose of link 0 (the fixed base), or NULL = identity
 *   q       device float [C][dof] joint angles (radians)
 *   link_T  device float [C][dof+1][3][4] output; link 0 is base_T, link k
 *           (1 <= k <= dof) is the frame after joint k
 * C = 0 enqueues nothing.  Computed in FP32. */
int lsdf_fk_batch(const lsdf_dh* dh, int32_t dof, const float* base_T,
                  const float* q, int32_t C, float* link_T, void* stream);

/* ---- clearance query -------------------------------------------------------
 * Sec. III-A: per configuration c, the minimum over obstacle points x_j and
 * links i of g_i(R_{i,c}^T (x_j - t_{i,c})), where g_i is the trilinear
 * interpolant of link i's grid inside its box and +infinity outside it.
 *   link_T        device float [C][L][3][4] link poses (e.g. from lsdf_fk_batch)
 *   grids         host [L] grid descriptors, 1 <= L <= LSDF_MAX_LINKS
 *   grid_buf      device buffer holding every link's grid
 *   points        device float [M][3] obstacle points (world frame)
 *   out_dist      device float [C]: the clearance (+inf when no point lies in
 *                 any link's box)
 *   out_link      device int32 [C]: lowest link index attaining out_dist, -1
 *                 when out_dist is +inf
 *   out_link_dist device float [C][L] per-link minima, or NULL
 *   flags         must be 0
 *   workspace     device scratch of at least lsdf_query_workspace_size()
 *                 bytes, 256-byte aligned.  Its contents on entry are
 *                 ignored (the call's first kernel initialises what it
 *                 uses) and are unspecified afterwards.  Calls that share a
 *                 workspace must not overlap in time (same stream is fine).
 * M <= LSDF_MAX_POINTS.  -0 is returned as +0.  M = 0 gives (+inf, -1) everywhere; C = 0 enqueues
 * nothing.  The arithmetic is FP32 in a fixed operation order (per link and
 * configuration the world-to-grid map is formed once as one affine matrix,
 * the form of Eq. 4; the lerp is fma(f, b, fma(-f, a, a))), so results are
 * reproducible bit for bit. */
/* Workspace bytes of a query of C configurations, L links and M points
 * with the given flags (the same flags the query will get; must be 0). */
int lsdf_query_workspace_size(int32_t C, int32_t L, int64_t M, uint32_t flags, size_t* bytes);

int lsdf_query_min_distance(const float* link_T, int32_t C, int32_t L,
                            const lsdf_grid* grids, const void* grid_buf,
                            const float* points, int64_t M,
                            float* out_dist, int32_t* out_link, float* out_link_dist,
                            uint32_t flags, void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, hosts that forbid allocation): lsdf_query_min_distance
 * with no workspace argument.  Its workspace is device memory the library
 * holds, LSDF_QUERY_NOALLOC_SCRATCH bytes on each GPU it runs on, from the
 * first call on that GPU until the process ends.  The call allocates
 * nothing.  Same arguments, kernels and results, bit for bit, as
 * lsdf_query_min_distance.  A problem whose workspace
 * (lsdf_query_workspace_size) exceeds that size is rejected with
 * LSDF_E_SHAPE before anything is enqueued; 8 MiB holds, for example, 500
 * configurations of 7 links with up to 3 million points.  Every call on one
 * GPU uses that GPU's one copy, so calls that overlap in time on one GPU
 * (different streams, or different host threads) race and give wrong
 * results; calls in one stream are ordered and safe.  The stream must belong
 * to the current device. */
#define LSDF_QUERY_NOALLOC_SCRATCH (((size_t)8) << 20)
int lsdf_query_min_distance_noalloc(const float* link_T, int32_t C, int32_t L,
                                    const lsdf_grid* grids, const void* grid_buf,
                                    const float* points, int64_t M,
                                    float* out_dist, int32_t* out_link, float* out_link_dist,
                                    uint32_t flags, void* stream);

/* ---- batched clearance query ----------------------------------------------
 * The same quantity for K trajectories in one call.  The paper re-plans a
 * path of a few hundred configurations against each new cloud, over and
 * over (Sec. IV); this call takes many such (path, cloud) pairs at once.
 * Trajectory k pairs configurations [c_off[k], c_off[k+1]) of link_T with
 * points [m_off[k], m_off[k+1]) of points; each configuration's result
 * is the plain query's over its own trajectory's points, bit for bit.
 *   K             number of trajectories, 1 <= K <= LSDF_MAX_TRAJECTORIES
 *   traj_c_offset DEVICE int32 [K+1], non-decreasing, in [0, C]
 *   traj_m_offset DEVICE int64 [K+1], non-decreasing, in [0, M]
 *   C, M          sizes of link_T / out_* and points (capacities: rows not
 *                 covered by any trajectory get (+inf, -1))
 *   tuning        work tiling, or NULL for the defaults (see below); it
 *                 changes the speed only, never a result bit
 *   other arguments as lsdf_query_min_distance; the workspace is sized by
 *   lsdf_query_batched_workspace_size(K, C, L, M) under the same rules.
 * The offsets are read on the device only, so the call copies nothing to or
 * from the host and can be captured in a HIP graph and replayed with new
 * offset, pose and point contents (same C, M, K capacities).  Offsets out
 * of order or out of range are clamped into [0, C] and [0, M] on the device:
 * the results are then meaningless, but no access leaves the buffers. */
#define LSDF_SCHED_DEFAULT     0   /* the library's choice (interleaved) */
#define LSDF_SCHED_XCD_SLICES  1   /* each XCD takes a contiguous slice of
                                      the work (its L2 sees few link grids) */
#define LSDF_SCHED_INTERLEAVED 2   /* every wave of the grid takes every W-th
                                      chunk (balances uneven work) */
typedef struct {
    int32_t chunk_points;   /* points per work chunk: a multiple of 8 in
                               [8, 8192], rounded up to a multiple of 32
                               (a chunk takes every n-th run of 32 points of
                               its trajectory's cloud); 0 = default (at
                               most about one chunk per wave of the grid
                               for C and M, 32 to 1024 points) */
    int32_t blocks_per_cu;  /* workgroups of the persistent grid per compute
                               unit, in [1, 16]; 0 = default (as many as fit
                               on a CU at once) */
    int32_t schedule;       /* LSDF_SCHED_* */
    int32_t reserved;       /* must be 0 */
} lsdf_query_tuning;

int lsdf_query_batched_workspace_size(int32_t K, int32_t C, int32_t L, int64_t M, size_t* bytes);

int lsdf_query_min_distance_batched(int32_t K, const int32_t* traj_c_offset, const int64_t* traj_m_offset,
                                    const float* link_T, int32_t C, int32_t L,
                                    const lsdf_grid* grids, const void* grid_buf,
                                    const float* points, int64_t M,
                                    float* out_dist, int32_t* out_link, float* out_link_dist,
                                    const lsdf_query_tuning* tuning, uint32_t flags,
                                    void* workspace, size_t ws_bytes, void* stream);

/* Kinematics and clearance in one call (Sec. III-A: forward kinematics of
 * every configuration, then the distance of each to the obstacles).  The
 * poses are computed in the query's first kernel, with the arithmetic of
 * lsdf_fk_batch (the same bits), which saves a launch per step.
 *   dh, dof, base_T   as lsdf_fk_batch; the grids are the dof + 1 frames'
 *   q                 device float [C][dof] joint angles
 *   K, traj_c_offset, traj_m_offset
 *                     as lsdf_query_min_distance_batched, or K = 1 with both
 *                     offset arrays NULL (one trajectory of all C and M)
 *   link_T            device float [C][dof+1][3][4] receiving the poses, or
 *                     NULL when only the clearances are wanted
 *   other arguments as lsdf_query_min_distance_batched (workspace sized by
 *   lsdf_query_batched_workspace_size(K, C, dof + 1, M)).
 * Results are bit-identical to lsdf_fk_batch followed by the query. */
int lsdf_query_from_joints(const lsdf_dh* dh, int32_t dof, const float* base_T, const float* q,
                           int32_t K, const int32_t* traj_c_offset, const int64_t* traj_m_offset,
                           int32_t C, const lsdf_grid* grids, const void* grid_buf,
                           const float* points, int64_t M, float* link_T,
                           float* out_dist, int32_t* out_link, float* out_link_dist,
                           const lsdf_query_tuning* tuning, uint32_t flags,
                           void* workspace, size_t ws_bytes, void* stream);

/* Picks the fastest tiling for one batched problem by timing it.
 * Runs lsdf_query_min_distance_batched once untimed and `reps` times timed
 * (HIP events on `stream`) per candidate, and returns the candidate with
 * the lowest mean time in *best (and that time in ms in *best_ms, which may
 * be NULL).  candidates = NULL uses a built-in list (the default tiling
 * first, then chunk_points 64 to 4096 on the resident grid, 4 workgroups per
 * CU, and per-XCD slices).  1 <= reps <= 1000.
 * It SYNCHRONISES the stream (not capturable); out_dist / out_link hold the
 * problem's results when it returns LSDF_OK. */
int lsdf_query_autotune(int32_t K, const int32_t* traj_c_offset, const int64_t* traj_m_offset,
                        const float* link_T, int32_t C, int32_t L,
                        const lsdf_grid* grids, const void* grid_buf,
                        const float* points, int64_t M, float* out_dist, int32_t* out_link,
                        const lsdf_query_tuning* candidates, int32_t n_candidates, int32_t reps,
                        void* workspace, size_t ws_bytes, void* stream,
                        lsdf_query_tuning* best, float* best_ms);

/* ---- the paper's Robot-SDF pipeline (comparator) ---------------------------
 * Sec. III-A, Eq. 1-4: per configuration, a Robot SDF over the voxels of
 * the environment (per voxel, the minimum over links of the link's SDF
 * transformed by its pose and aligned to the voxel grid), then at run time
 * the distance of each configuration is the minimum of its Robot SDF over
 * the voxels the obstacle points occupy.  The per-point query above is the
 * library's method; these calls reproduce the paper's for comparison (its
 * trade-off: C x V voxels of memory and a heavy preparation against a
 * gather-only runtime).
 * The environment: voxel v (0 <= v_a < n_a) spans [lo_a + v_a r,
 * lo_a + (v_a + 1) r) (lo = -e_e, the paper's extent; r = voxel, its
 * resolution).  Link i's block at configuration c covers voxels k .. k + 2m
 * - 1 per axis with k = round((t - lo) / r) - m (Eq. 1-2 in double, t the
 * link origin) and m = ceil(farthest grid-box corner from the link origin
 * / r) + 2.  A voxel's value is the minimum, over the links whose block
 * covers it, of the link grid's interpolant at the voxel centre
 * lo + (v + 1/2) r (double, rounded once to float) moved into the link frame
 * (Eq. 4), with the plain query's FP32 arithmetic (so each value equals the
 * plain query at that point), +inf where none applies. */
typedef struct {
    float lo[3];      /* environment corner, metres */
    float voxel;      /* voxel edge r > 0, metres */
    int32_t n[3];     /* voxels per axis, 1..4096, at most 2^32 in all */
} lsdf_env;

/* Bytes of the Robot SDFs of C configurations: C * n_x * n_y * n_z * 4. */
int lsdf_robot_sdf_size(int32_t C, const lsdf_env* env, size_t* bytes);
int lsdf_robot_sdf_build_workspace_size(int32_t C, int32_t L, size_t* bytes);

/* Preparation: fills robot_sdf, device float [C][n_z][n_y][n_x] (x
 * fastest), from link poses link_T [C][L][3][4] and the link grids.  Every
 * voxel is written.  workspace: device, 256-byte aligned, at least
 * lsdf_robot_sdf_build_workspace_size(C, L) bytes; contents ignored. */
int lsdf_robot_sdf_build(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                         const void* grid_buf, const lsdf_env* env, float* robot_sdf,
                         void* workspace, size_t ws_bytes, void* stream);

int lsdf_robot_sdf_query_workspace_size(const lsdf_env* env, int64_t M, size_t* bytes);

/* Runtime: out_dist[c] = minimum of robot_sdf[c] over the distinct voxels
 * holding at least one of the points (voxel of x: floor((x - lo) / r),
 * in double; points outside the environment are ignored); +inf when no
 * point is inside.  workspace: device, 256-byte aligned, at least
 * lsdf_robot_sdf_query_workspace_size(env, M) bytes; contents ignored.
 * When the call's work has completed, the workspace holds the distinct
 * occupied voxels for inspection: with V = n[0] n[1] n[2] and
 * K = 256 * ceil(4 * ceil(V / 32) / 256), their count as a uint32 at byte
 * K, and their flat indices (uint32, in no particular order) from byte
 * K + 256 on. */
int lsdf_robot_sdf_query(const float* robot_sdf, int32_t C, const lsdf_env* env,
                         const float* points, int64_t M, float* out_dist,
                         void* workspace, size_t ws_bytes, void* stream);

/* ---- the paper's grid-transformation network f(R) -------------------------
 * Sec. III-B-1, Eq. 4-5: a tiny network maps a link rotation R to the
 * rotated, normalised centres of the (2m)^3 voxels of a transformed Link
 * SDF block, f(R) ~ R^T P_j with P_j = (j + 1/2) / m - 1 per axis; the
 * block's link-frame points are then e_r (f(R) - R^T dt / e_r), e_r = m r.
 *   x = R row-major (9), h = ReLU(W1 x + b1) (LSDF_FRNN_HIDDEN units),
 *   out = W2 h + b2 (3 V outputs, V = (2m)^3, output 3 j + a for voxel
 *   j = (j_z 2m + j_y) 2m + j_x and axis a).
 * Parameters (FP32, device): W1[H][9], b1[H], W2[3V][H], b2[3V], H = 32;
 * lsdf_frnn_nparam gives their count.  1 <= m <= LSDF_FRNN_MAX_HALF. */
int lsdf_frnn_nparam(int32_t m, int64_t* n);
int lsdf_frnn_train_workspace_size(int32_t m, int32_t B, size_t* bytes);

/* One training step on B rotations R (device float [B][9], 1 <= B <= 64):
 * the mean absolute error against R^T P over the batch and every output
 * (the paper's L1 loss, Sec. IV-B) into loss_out (device float [1], may be
 * NULL), its gradient into grad (device float [n]), then, when adam_m and
 * adam_v (device float [n]) are given, one Adam update of params with step
 * t >= 1 (bias-corrected).  With adam_m = adam_v = NULL only the loss and
 * the gradient are computed.  FP32; deterministic (no float atomics). */
int lsdf_frnn_train_step(float* params, float* adam_m, float* adam_v, int64_t t, float lr,
                         float beta1, float beta2, float eps, int32_t m, const float* R, int32_t B,
                         float* loss_out, float* grad, void* workspace, size_t ws_bytes, void* stream);

/* max over N rotations (device float [N][9]) and all 3V outputs of
 * |f(R) - R^T P| into out_max (device float [1]): the paper's test of the
 * approximation over 10^7 random transformations (Sec. IV-B). */
int lsdf_frnn_max_error(const float* params, int32_t m, const float* R, int64_t N, float* out_max,
                        void* stream);

/* lsdf_robot_sdf_build with the transformation taken from the network
 * (Eq. 5) instead of computed exactly: every link uses the network's block
 * half-width m (which must hold each link's grid box, else LSDF_E_SHAPE);
 * block voxel j of link i at configuration c is read at the link-frame point
 * e_r (f(R)_j - R^T dt / e_r).  Values are approximate (the network's
 * error times e_r). */
int lsdf_robot_sdf_build_frnn(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                              const void* grid_buf, const lsdf_env* env, const float* frnn_params,
                              int32_t m, float* robot_sdf, void* workspace, size_t ws_bytes, void* stream);

/* ---- link SDF construction -------------------------------------------------
 * Sec. III-A: each link's signed distance field is computed once, offline,
 * on a grid in the link's own frame.  The paper does not say how; this call
 * uses the brute-force exact signed distance to a closed triangle mesh.
 *   verts       device float [nv][3] vertices in the link frame
 *   tris        device int32 [nt][3] triangles, outward (counter-clockwise)
 *   comp_first  host int32 [ncomp+1]: triangles [comp_first[k],
 *               comp_first[k+1]) form closed part k; NULL = one part of all
 *               nt triangles.  The link's distance is the minimum over parts.
 *   desc        host descriptor of the grid to fill; 16-bit storage holds the
 *               FP32 distance rounded once to nearest even
 *   grid_buf    device buffer; nodes are written at desc->elem_offset
 * Inside/outside is decided by the generalised winding number of each part
 * (negative inside). */
int lsdf_build_link_sdf(const float* verts, int32_t nv, const int32_t* tris, int32_t nt,
                        const int32_t* comp_first, int32_t ncomp, const lsdf_grid* desc,
                        void* grid_buf, void* stream);

/* ---- learned per-link SDF surrogate ---------------------------------------
 * An extension of the method (not in the paper): per link, a small network
 * m(x) = w4 . h3 + b4, h_k = SiLU(W_k h_{k-1} + b_k), widths 3 -> 128 -> 128
 * -> 128 -> 1, SiLU(z) = z / (1 + exp(-z)), maps a link-frame point l
 * normalised to the link's domain to the remainder of the link's signed
 * distance over E(l), the distance from l to the link's core box (its mesh's
 * bounding box); the estimate is E + B tanh(m / B) with the link's remainder
 * bound B (B = +inf: E + m).  E carries the distance's growth far from the
 * link, so the network only fits a bounded, slowly varying remainder, and
 * since the estimate lies within B of E a query skips, exactly, the points
 * that cannot hold a link's minimum.  It answers queries beyond the grid box
 * (the far field); the grid stays the answer for every pair in the box whose
 * estimate is below a safety margin.  The paper's own network
 * (Sec. III-B-1) is a different one (it approximates the grid transform);
 * its training recipe (L1 loss, Adam, Sec. IV-B) is reused here.
 *
 * Parameters: FP32 [L][LSDF_MLP_PARAMS] per link, laid out as
 * W1[128][3], b1[128], W2[128][128], b2[128], W3[128][128], b3[128],
 * w4[128], b4 (row-major [out][in]).  W1, W2, W3 and w4 are used rounded to
 * bfloat16 (nearest even); activations are rounded to bfloat16 before each
 * product; the input layer runs in FP32 and the 128x128 layers on bf16 MFMA
 * with FP32 accumulation. */
#define LSDF_MLP_HIDDEN 128
#define LSDF_MLP_PARAMS 33665

/* Normalisation of a link's network input: xhat = (x_link - centre) / half;
 * the domain is |xhat_a| <= 1 on every axis.  The core box is
 * |x_link - centre| <= core_half on every axis; its distance
 * E = || max(|x_link - centre| - core_half, 0) || (FP32: u = x_link - centre,
 * q = max(|u| - core_half, 0), E = sqrt(fma(qx, qx, fma(qy, qy, qz * qz))),
 * correctly rounded) is added to the network's share, which is
 * bound * t with t = clamp(1 - 2 / (1 + exp(2 m / bound)), -1, 1) (in FP32,
 * m times (float)(1 / bound)), or m itself when bound = +inf. */
typedef struct lsdf_mlp_domain {
    float centre[3];
    float half[3];       /* each > 0 */
    float core_half[3];  /* each >= 0 */
    float bound;         /* > 0, or +inf */
} lsdf_mlp_domain;

/* The surrogate's estimates (bounded network share + core distance) at N
 * link-frame points of one link.
 *   params  device float [LSDF_MLP_PARAMS]; domain host; points device [N][3];
 *   out     device float [N] (evaluated also outside the domain). */
int lsdf_mlp_eval(const float* params, const lsdf_mlp_domain* domain, const float* points, int64_t N,
                  float* out, void* stream);

/* Clearance with the learned surrogate: as lsdf_query_min_distance, but the
 * value of pair (c, i, j) is m = the estimate of link i at the point (bounded
 * network share + core distance) if the point lies in link i's domain (the
 * pair is skipped otherwise), replaced by
 * the grid value when m < margin (strict) and the point lies in link i's grid
 * box.  A point outside the box keeps m whatever its value, since the grid
 * has no value there (when the box pads the link's bounding box by at least
 * the margin, such an m below the margin underestimates the distance).  Same
 * workspace as lsdf_query_min_distance
 * (lsdf_query_workspace_size).  margin may be +inf (every in-box pair takes
 * the grid value) or -inf (none does).  A pair that takes the grid value gets
 * exactly the bits lsdf_query_min_distance would give it.  With a finite
 * bound B_i a first kernel finds, per (c, i), U = the smallest E + B_i over
 * a sample of the in-domain pairs with E - B_i >= margin (pairs that cannot
 * fall back; the sample: the first point of every 32-point tile), and the
 * network is evaluated only for 32-pair tiles (or the 16-pair half of one)
 * holding a pair with
 * E - B_i <= max(min(U, the smallest value found so far), margin): every
 * other pair's value exceeds a value some pair has, so the per-link minima
 * are those of evaluating every pair. */
int lsdf_query_min_distance_mlp(const float* link_T, int32_t C, int32_t L, const lsdf_grid* grids,
                                const void* grid_buf, const float* mlp_params, const lsdf_mlp_domain* domains,
                                float margin, const float* points, int64_t M, float* out_dist, int32_t* out_link,
                                float* out_link_dist, uint32_t flags, void* workspace, size_t ws_bytes,
                                void* stream);

/* Training.  For each link i, B samples are taken from that link's N
 * samples (link-frame points [L][N][3] with labels [L][N]) through
 * batch_index [L][B] (NULL = the first B), and the mean absolute error of
 * the estimate (bounded network share + core distance) over them is
 * differentiated
 * (Sec. IV-B trains with an L1 loss).
 *   lsdf_mlp_loss_grad: loss_out [L] (or NULL), grad_out [L][LSDF_MLP_PARAMS]
 *   lsdf_mlp_train_step: the same, then one Adam step (Kingma & Ba) on
 *     params with moments adam_m, adam_v (FP32, same shape, zero at t = 1),
 *     step t >= 1; grad_out may be NULL.
 * B must be a positive multiple of 512.  The workspace (any contents) has at
 * least lsdf_mlp_train_workspace_size() bytes, 256-byte aligned. */
int lsdf_mlp_train_workspace_size(int32_t L, int32_t B, size_t* bytes);
int lsdf_mlp_loss_grad(const float* params, const lsdf_mlp_domain* domains, int32_t L, const float* samples,
                       const float* labels, int64_t N, const int32_t* batch_index, int32_t B, float* loss_out,
                       float* grad_out, void* workspace, size_t ws_bytes, void* stream);
int lsdf_mlp_train_step(float* params, float* adam_m, float* adam_v, int64_t t, float lr, float beta1, float beta2,
                        float eps, const lsdf_mlp_domain* domains, int32_t L, const float* samples,
                        const float* labels, int64_t N, const int32_t* batch_index, int32_t B, float* loss_out,
                        float* grad_out, void* workspace, size_t ws_bytes, void* stream);

/* Training labels at N link-frame points of one link: the grid value
 * (lsdf_query_min_distance's arithmetic, identity pose) inside the grid box,
 * the exact signed distance to the mesh outside it (brute force, as in
 * lsdf_build_link_sdf).  Arguments as in lsdf_build_link_sdf; points device
 * [N][3], out device [N]. */
int lsdf_sdf_labels(const float* verts, int32_t nv, const int32_t* tris, int32_t nt, const int32_t* comp_first,
                    int32_t ncomp, const lsdf_grid* desc, const void* grid_buf, const float* points, int64_t N,
                    float* out, void* stream);

/* Measurement aid, not part of the query path: `threads` threads each take
 * `iters` random cells of an n^3 FP32 grid (device, n^3 floats, x fastest,
 * cells drawn by a counter-based hash of thread and iteration) and sum the
 * cell's 8 corners, the gather of one trilinear sample; out (device
 * [threads]) receives each thread's sum.  Timing a launch gives the gather
 * rate a grid of that size sustains.  2 <= n <= 1024, iters >= 1,
 * 1 <= threads <= 2^31. */
int lsdf_gather_roof(const float* grid, int32_t n, int32_t iters, int64_t threads, float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LSDF_H */
