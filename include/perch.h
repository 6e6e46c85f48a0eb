/*
 * perch.h -- C ABI of the MI355X pose-scoring library (libperch.so).
 *
 * The library scores candidate 6-DoF object poses against an observed RGB-D
 * scene with the explanation cost of PERCH 2.0 (Agarwal, Han, Likhachev):
 *   J = J_r + J_o                                      (Sec. III-B, Eq. 1)
 *   J_r = rendered points, minus the occluded ones, with no observed point
 *         within delta                                 (Eq. 2, Eq. 3)
 *   J_o = observed points inside the object's volume with no rendered point
 *         within delta                                 (Eq. 2, Eq. 3)
 * and, with the RGB term, a point whose nearest neighbour lies within delta
 * is still an outlier when their CIEDE2000 colour difference exceeds tau_c
 * (Sec. IV-B, Eq. 4).  Each pose is rendered into depth (and colour) and
 * back-projected to points (Sec. IV-A "Parallel Rendering"); the best pose of
 * each object is the one of minimum cost (Sec. IV-A "Parallel Search").
 *
 * Conventions shared by every entry point:
 *  - Every call returns a perch_status; PERCH_OK is 0.  On error nothing is
 *    launched, no state changes, and perch_last_error() (thread-local) holds
 *    a message.  No C++ exception crosses the ABI.
 *  - Lengths are millimetres.  A pose is 12 binary32 values, row-major
 *    [R | t], mapping object coordinates to camera coordinates (x right,
 *    y down, z forward).  Intrinsics follow the pinhole model, and integer
 *    pixel coordinates are pixel centres.
 *  - Pointers named *_dev are device memory owned by the caller; they must
 *    stay valid until the work queued on the given stream has completed.
 *    Host pointers are read during the call only.
 *  - Results are deterministic: the same inputs give bit-identical outputs,
 *    whatever else is queued on the device.
 *  - A context belongs to one device.  Calls on one context may come from
 *    several threads and are serialised internally, but the waits inside
 *    perch_set_scene, perch_best_poses and perch_batch_wait are made outside
 *    that lock, so one thread can prepare a scene while another waits for
 *    scores.  A stream or a batch is used by one thread at a time.
 *  - Device memory released by perch_drop_scene / perch_unload_mesh is kept
 *    by the context and reused once every launch enqueued through it that
 *    reads the released scene or mesh has completed; neither call waits.
 *
 * Geometry, depth, coverage, point coordinates and all depth-only counts are
 * exact integers (8 sub-pixel bits, top-left fill rule, 16-bit millimetre
 * depth buffer, points in 1/16 mm).  The colour decision is taken in binary32
 * CIELAB/CIEDE2000.
 */
#ifndef PERCH_H
#define PERCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PERCH_OK = 0,
    PERCH_EINVAL = -1,    /* bad argument: sizes, indices, flags, null pointers */
    PERCH_ENOMEM = -2,    /* the context's HBM budget (or the device) is exhausted */
    PERCH_EDEVICE = -3,   /* a HIP runtime call failed */
    PERCH_ENOTFOUND = -4, /* unknown mesh or scene id */
    PERCH_EBUSY = -5      /* the object is in use (e.g. unload while queued) */
} perch_status;

typedef struct perch_ctx perch_ctx;

/* Scene flags. */
#define PERCH_USE_RGB 1u           /* Eq. 4 colour term (needs scene and mesh colours) */
#define PERCH_MARK_OCCLUDERS 2u    /* Eq. 3 occluders C from the observed depth */
#define PERCH_VOL_AABB (0u << 4)   /* V(O): object-frame mesh AABB inflated by delta */
#define PERCH_VOL_CYL (1u << 4)    /* V(O): cylinder about the object z axis through the centre of the
                                    * AABB's xy extent, radius the smaller xy half-extent plus delta,
                                    * z range of the AABB inflated by delta (Table I's conservative
                                    * volume taken as an inscribed cylinder) */
#define PERCH_VOL_LABEL (2u << 4)  /* V(O): observed pixels carrying the object's label (Sec. V-C) */
#define PERCH_VOL_MASK (3u << 4)
#define PERCH_JO_NN (1u << 6)      /* J_o by nearest-neighbour marking (Sec. IV-A, parallel cost
                                    * computation): an observed point of V(O) is explained only when it
                                    * is the nearest observed neighbour of a rendered inlier that passed
                                    * the colour test; without it, any rendered point within delta (with
                                    * a matching colour, Eq. 4) explains it, as Eq. 3 states */
#define PERCH_KNN2 (1u << 7)       /* J_r's nearest observed neighbours by the paper's kNN II search
                                    * (Sec. IV-A): each rendered point scans the whole observed cloud
                                    * instead of reading the scene's neighbour table.  Same results;
                                    * orders of magnitude slower (an in-house comparison baseline) */
#define PERCH_HASH (1u << 9)       /* J_r's nearest observed neighbours through a uniform-grid voxel
                                    * hash of the observed cloud (the search structure for the radius
                                    * test of Eq. 2; the CPU original searched a k-d tree per cloud):
                                    * cells of edge 2^k >= delta (1/16 mm units), cell coordinates
                                    * hashed into 2^m buckets (2^m >= 2 W H), the points of each bucket
                                    * stored contiguously (count, exclusive scan, scatter at set-up);
                                    * a query scans the buckets of the 27 cells around its point.  The
                                    * scene then holds no nearest-neighbour table (a fraction of the
                                    * device memory); results are identical, ties to the lower pixel
                                    * index as everywhere.  Not combined with PERCH_KNN1 / PERCH_KNN2 */
#define PERCH_KNN1 (1u << 8)       /* Both searches by the paper's kNN I (Sec. IV-A): every distance
                                    * between a pose's rendered points and the observed cloud goes
                                    * into one L x I array (4 bytes a pair) that is then reduced by
                                    * rows (J_r) and by columns (J_o).  Same results as the table;
                                    * one pose at a time, a comparison baseline scored by
                                    * perch_score_poses only (refused by the batched, best-pose and
                                    * tree entry points); not combined with PERCH_KNN2 */

typedef struct {
    int32_t width, height;   /* pixels, 1 .. 4096 */
    float fx, fy, cx, cy;    /* fx, fy > 0 */
} perch_intrinsics;

typedef struct {
    perch_intrinsics K;
    const uint16_t *depth_mm; /* H*W row-major host array, 0 = no reading (required) */
    const uint8_t *rgb;       /* H*W*3 sRGB8 host array, or NULL (depth only) */
    const int32_t *labels;    /* H*W host array, or NULL (required for PERCH_VOL_LABEL) */
    float delta_mm;           /* sensor resolution delta, 0 < delta <= 500 */
    float tau_c;              /* CIEDE2000 threshold tau_c >= 0, used with PERCH_USE_RGB */
    uint32_t flags;           /* PERCH_USE_RGB | PERCH_MARK_OCCLUDERS | PERCH_VOL_* | PERCH_JO_NN | PERCH_KNN2 |
                                 PERCH_KNN1 | PERCH_HASH */
    int32_t stride;           /* image-space downsampling of the render, >= 1 (Sec. IV-A) */
} perch_scene_desc;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory held for meshes, scenes and work buffers (0 = no cap).  The context
 * owns one HIP stream on which it prepares scenes.  Every call that takes a
 * hip_stream enqueues on that stream; NULL means the HIP null stream. */
perch_status perch_create(int device, size_t hbm_budget_bytes, perch_ctx **out);

/* Release every mesh, scene and buffer of the context, after waiting for its
 * queued work.  A NULL context is accepted. */
perch_status perch_destroy(perch_ctx *ctx);

/* Copy a triangle mesh to the device (the object model of Sec. III-A).
 * xyz_mm: n_verts*3 binary32, object frame.  tri: n_tris*3 vertex indices,
 * counter-clockwise about the outward normal (back faces are culled).
 * rgb: n_verts*3 sRGB8 per-vertex colours, or NULL.  1 <= n_tris <= 65535. */
perch_status perch_load_mesh(perch_ctx *ctx, const float *xyz_mm, int32_t n_verts,
                             const int32_t *tri, int32_t n_tris, const uint8_t *rgb,
                             int32_t *mesh_id);
perch_status perch_unload_mesh(perch_ctx *ctx, int32_t mesh_id);

/* Copy an observed RGB-D image to the device and prepare it for scoring (the
 * input cloud I of Sec. III-B): back-projection to points in 1/16 mm, CIELAB
 * colours, and a nearest-neighbour table -- for every pixel and every depth
 * a rendered point there could have, the nearest observed point within
 * delta (Eq. 2), ties to the lower pixel index.  Returns when the scene is
 * ready; the preparation runs on the context's own stream.  The table is
 * allocated at its exact size: counted by the device (one wait for the
 * count), or, while a batch of this context is running, by the host (the
 * device's count is then checked against it: PERCH_EDEVICE on a difference). */
perch_status perch_set_scene(perch_ctx *ctx, const perch_scene_desc *desc, int32_t *scene_id);
perch_status perch_drop_scene(perch_ctx *ctx, int32_t scene_id);

typedef struct {
    size_t device_bytes;          /* HBM held by the scene (images, points, neighbour table) */
    int64_t table_entries;        /* entries of its nearest-neighbour table */
    int32_t window_x, window_y;   /* pixel half-windows that contain every neighbour pair */
    int32_t tile_cap_small;       /* LDS words (raster tile + J_o keys) of the scoring classes */
    int32_t tile_cap_large;       /*   1 and 2; larger footprints use device memory */
    int32_t table_counted_on_host; /* 1 when the table's size was counted on the host */
    int32_t reserved;
} perch_scene_info;

/* Describe a resident scene (footprint, search windows, tile classes). */
perch_status perch_scene_info_get(perch_ctx *ctx, int32_t scene_id, perch_scene_info *out);

/* Entries of a neighbour table as set_scene counts them on the host (host
 * code only; no device is used): for every pixel of the w x h depth image
 * (uint16 mm, 0 = no reading; host memory, read only) the depths
 * [min - dzmm, max + dzmm], kept inside [1, 65534], of the valid readings in
 * its window of (2 wx + 1) x (2 wy + 1) pixels clipped to the image, and
 * none where the window holds no reading.  *entries receives the sum, or -1
 * when wx or wy exceeds 48 (set_scene then lets the device count).
 * PERCH_EINVAL on null pointers, w or h < 1, or wx, wy, dzmm < 0. */
perch_status perch_table_entries(const uint16_t *depth_mm, int32_t w, int32_t h, int32_t wx, int32_t wy,
                                 int32_t dzmm, int64_t *entries);

/* Score n poses of one mesh in one scene (Eq. 3 / Eq. 4).  Asynchronous on
 * hip_stream.
 *   label:      the object's label; used by PERCH_VOL_LABEL and, in that
 *               mode, to keep same-label pixels from occluding (Sec. V-C).
 *   poses_dev:  n*12 binary32 device array.
 *   jr_dev, jo_dev: n int32 device arrays, J_r and J_o per pose.
 *   nr_dev, nq_dev: n int32 device arrays or NULL: L = |R \ C| and
 *               Q = |I inside V(O)| per pose.
 * n may be 0 (nothing is launched). */
perch_status perch_score_poses(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                               const float *poses_dev, int32_t n, int32_t *jr_dev,
                               int32_t *jo_dev, int32_t *nr_dev, int32_t *nq_dev,
                               void *hip_stream);

/* perch_score_poses with the decision behind every count (Eq. 3, Eq. 4),
 * for inspection and testing: the same kernels score the n poses and also
 * write, per pose, two H*W uint8 images (device, caller-owned, n*H*W bytes
 * each, cleared by the call):
 *   rflag_dev: each rendered pixel -- 0 not in R (empty or off the stride
 *              grid), 1 inlier, 2 no observed point within delta, 3 nearest
 *              observed point within delta but CIEDE2000 above tau_c,
 *              4 occluder (dropped, Eq. 3's C)
 *   oflag_dev: each observed pixel -- 0 outside V(O), 1 explained, 2 no
 *              rendered point within delta, 3 nearest rendered point within
 *              delta but CIEDE2000 above tau_c (with PERCH_JO_NN: 1 marked,
 *              2 not)
 * 1 <= n <= 256.  Asynchronous on hip_stream; PERCH_KNN1 scenes are refused. */
perch_status perch_score_detail(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                                const float *poses_dev, int32_t n, int32_t *jr_dev, int32_t *jo_dev,
                                int32_t *nr_dev, int32_t *nq_dev, uint8_t *rflag_dev, uint8_t *oflag_dev,
                                void *hip_stream);

/* perch_score_poses for callers that cannot allocate memory (code that may
 * be captured into a HIP graph, tight serving loops, hosts that forbid
 * allocation during a request): the same kernels, with every launch buffer
 * -- descriptors, per-pose work, class lists, counters and the device-memory
 * slots of the largest footprints -- carved from one 48 MiB array that each
 * device holds for the life of the process.  The call allocates no device
 * or host-pinned memory; the caller passes poses and outputs as for
 * perch_score_poses, and the outputs are bit-identical to its.
 * Limits: 0 <= n <= 65536 poses, scenes of at most 640 * 480 pixels, no
 * PERCH_KNN1 scenes; beyond them PERCH_EINVAL and nothing is launched.
 * Every call on a device, from any context of the process, shares that
 * device's array and the last call leaves its contents there: two calls
 * whose device work overlaps (different streams without an ordering
 * between them) race and their results are undefined.  Calls queued on one
 * stream are ordered and safe.  Asynchronous on hip_stream. */
perch_status perch_score_poses_noalloc(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                                       const float *poses_dev, int32_t n, int32_t *jr_dev, int32_t *jo_dev,
                                       int32_t *nr_dev, int32_t *nq_dev, void *hip_stream);

/* One slice of a launch: the candidate poses of one object in one scene.
 * Pointers as in perch_score_poses; n_poses may be 0. */
typedef struct {
    int32_t scene_id, mesh_id, label, n_poses;
    const float *poses_dev;        /* n_poses * 12 binary32 */
    int32_t *jr_dev, *jo_dev;      /* n_poses each */
    int32_t *nr_dev, *nq_dev;      /* n_poses each, or NULL */
} perch_work;

/* Score many (scene, object, poses) items -- any mix of resident scenes and
 * meshes -- in one launch sequence on hip_stream; asynchronous.  Each item's
 * outputs are bit-identical to scoring it alone with perch_score_poses. */
perch_status perch_score_batch(perch_ctx *ctx, const perch_work *items, int32_t n_items, void *hip_stream);

/* A prepared batch: buffers for up to max_items items holding max_poses poses
 * in total, in scenes of at most max_image_pixels pixels, and a captured HIP
 * graph (descriptor upload, scoring, per-item minimum, result download).
 * perch_batch_set writes the work descriptors (waiting for a previous launch
 * of the batch to finish); perch_batch_launch replays the graph on
 * hip_stream; perch_batch_wait blocks and returns, per item, the minimum-cost
 * pose index and its J (-1 for items without poses).  Items' J_r / J_o
 * arrays are filled as in perch_score_batch.  Scenes and meshes named by a
 * set batch must stay resident: dropping one while a launch is pending
 * returns PERCH_EBUSY, otherwise it invalidates the batch until the next set. */
typedef struct perch_batch perch_batch;
perch_status perch_batch_create(perch_ctx *ctx, int32_t max_items, int32_t max_poses, int32_t max_image_pixels,
                                perch_batch **out);
perch_status perch_batch_set(perch_batch *batch, const perch_work *items, int32_t n_items);
perch_status perch_batch_launch(perch_batch *batch, void *hip_stream);
perch_status perch_batch_wait(perch_batch *batch, int32_t *best_idx_host, int32_t *best_cost_host);
/* Non-blocking: PERCH_OK when the batch's last launch has finished (or it
 * was never launched), PERCH_EBUSY while it is still running. */
perch_status perch_batch_query(perch_batch *batch);
perch_status perch_batch_destroy(perch_batch *batch);

/* Minimum-cost pose of each of n_obj objects (Sec. IV-A "Parallel Search"):
 * scores every candidate and reduces J = J_r + J_o per object on the device;
 * ties go to the lowest pose index.  Blocks until the results are on the
 * host.  mesh_ids, labels, n_poses: n_obj host arrays; poses_dev: n_obj host
 * pointers to device pose arrays.  best_idx_host, best_cost_host: n_obj host
 * outputs.  Every n_poses[k] must be >= 1. */
perch_status perch_best_poses(perch_ctx *ctx, int32_t scene_id, int32_t n_obj,
                              const int32_t *mesh_ids, const int32_t *labels,
                              const float *const *poses_dev, const int32_t *n_poses,
                              int32_t *best_idx_host, int32_t *best_cost_host,
                              void *hip_stream);

/* Render n poses of a mesh with the scene's camera into full images, with
 * the same rasterizer the scorer uses (Sec. IV-A "Parallel Rendering"):
 * depth_dev n*H*W uint16 (0 = empty), rgb_dev n*H*W*3 uint8 or NULL (needs
 * mesh colours), tri_dev n*H*W int32 winning triangle (-1 = empty) or NULL.
 * Asynchronous; 1 <= n <= 256.  Meant for inspection and testing. */
perch_status perch_render(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id,
                          const float *poses_dev, int32_t n, uint16_t *depth_dev,
                          uint8_t *rgb_dev, int32_t *tri_dev, void *hip_stream);

/* ICP refinement parameters (perch_refine_poses). */
typedef struct {
    int32_t iterations;   /* at most this many updates, 1 .. 1000 */
    float max_corr_mm;    /* correspondence radius rho, 0 < rho <= 100 mm */
    int32_t stride;       /* image-space downsampling of the rendered (source) cloud, >= 1 */
    int32_t dof;          /* 3: rotation about the pose's object z axis and translation normal to it
                           *    (the 3-DoF table-top search); 6: any rigid motion */
    int32_t min_points;   /* stop when fewer points match, >= 3 */
    int32_t method;       /* PERCH_ICP_POINT or PERCH_ICP_PLANE (GICP; needs dof 6) */
} perch_icp_params;

#define PERCH_ICP_POINT 0   /* point-to-point: the update aligns the matched pairs */
#define PERCH_ICP_PLANE 1   /* plane-to-plane GICP (Sec. IV-A "Parallel M2M GICP"): each point's
                             * surface a Gaussian, covariance I - (1 - 1/1024) n n^T with the normal n
                             * from the cross product of its pixel neighbours' points (none at depth
                             * steps over floor(rho) mm: covariance I); one Gauss-Newton step of the
                             * rigid motion about the matches' rounded centre per iteration, its terms
                             * summed exactly in 64-bit fixed point (times 1024), solved by Cholesky */

/* ICP refinement of candidate poses (Sec. IV-A "Parallel M2M GICP"; the
 * point-to-point ICP of the 3-DoF experiments, Sec. VI-A), the step before
 * rendering and scoring the adjusted poses again.  Per pose: the rendered
 * points that the scorer keeps (occluders removed as the scene's flags say,
 * here on the ICP stride grid) are aligned to the observed cloud — with
 * PERCH_VOL_LABEL, to the observed pixels carrying `label` (Sec. V-C).  Each
 * iteration maps them by the current camera-frame transform, rounded to
 * 1/16 mm; matches each with its nearest observed point within rho (ties:
 * lower pixel index; exact integers); sums the pairs exactly; and takes
 * the update about the source centroid.  For 3-DoF that is the planar
 * least-squares rotation about the axis and the in-plane translation; for
 * 6-DoF, one Gauss-Newton step of the linearised rotation, applied as a unit
 * quaternion.  ICP stops after `iterations` updates, when fewer than
 * min_points match, when no mapped point moved, or (6-DoF) on a singular
 * system.
 *   poses_dev:   n*12 binary32 [R|t] object -> camera, mm (device, read)
 *   refined_dev: n*12 binary32 refined poses (device, written; may not alias
 *                poses_dev)
 *   iters_dev:   n int32 updates applied, or NULL
 *   matched_dev: n int32 matches in the last iteration examined, or NULL
 * Asynchronous on hip_stream.  Device scratch of the stream: a W*H tile and
 * 2*W*H points per work-group (one per compute unit, at most n). */
perch_status perch_refine_poses(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                                const float *poses_dev, int32_t n, const perch_icp_params *params,
                                float *refined_dev, int32_t *iters_dev, int32_t *matched_dev,
                                void *hip_stream);

/* 6-DoF pose proposal parameters (perch_propose_poses). */
typedef struct {
    int32_t viewpoints;   /* M >= 1 viewpoints on the unit sphere */
    int32_t inplane;      /* N >= 1 in-plane angles 2 pi k / N */
    float z_step_mm;      /* spacing of the depth proposals, > 0 */
    int32_t max_depths;   /* at most this many depths T >= 1 (then spread evenly over the range) */
} perch_proposal_params;

/* 6-DoF pose proposals of one object (Sec. V-B "Pose Proposal Generation"):
 * every combination of M rotation viewpoints, N in-plane angles and T depths,
 * pose p = (i N + k) T + t.  Viewpoint i sits on the Fibonacci lattice of
 * the unit sphere (z = 1 - (2i + 1)/M, longitude i pi (3 - sqrt 5)): the
 * nearest to equidistant for any M; the rotation turns it to face the
 * camera, then by 2 pi k / N about the optical axis.  The translation puts
 * the object's centre (the centre of the mesh's object-frame AABB) on the
 * ray through the centre of the label's pixel box (the scene's labels stand
 * in for the segmentation masks) at depth
 * z_t = z_min + t * z_step_mm, with [z_min, z_max] the range of valid
 * observed depths under the label; when that gives more than max_depths,
 * T = max_depths depths spread evenly over the range.  Needs scene labels.
 *   poses_dev: capacity*12 binary32 (device, written), or NULL to count only
 *   n_out:     host int32, the number of proposals M*N*T (0 when the label
 *              has no pixel with a depth reading)
 * Asynchronous on hip_stream; PERCH_EINVAL when capacity < M*N*T. */
perch_status perch_propose_poses(perch_ctx *ctx, int32_t scene_id, int32_t mesh_id, int32_t label,
                                 const perch_proposal_params *params, float *poses_dev,
                                 int32_t capacity, int32_t *n_out, void *hip_stream);

/* Monotone Scene Generation tree (the sequential search of the original
 * PERCH that the variant 2.0-B of PERCH 2.0 keeps, Sec. III-B and its tree
 * figure, Sec. VI-A).  A state is a sequence of placed objects; its render
 * is their renders composed in order (a pixel keeps the first object that
 * draws it).  A successor appends one object in one candidate pose and is
 * monotone iff that object is nearer than the state's render on no pixel
 * both draw.  Its edge cost is J_r over the object's own points dR (its
 * pixels the state leaves empty, on the stride grid, less occluders) plus
 * J_o over the observed points inside its volume V(O) and inside no placed
 * object's volume, each tested against the composed render's points R \ C
 * (Eq. 3, Eq. 4).  Nearest-neighbour J_o marking (PERCH_JO_NN) and PERCH_KNN1
 * scenes are refused; PERCH_KNN2 does not apply (the scene's table gives the
 * same neighbours). */
typedef struct {
    int32_t mesh_id, label;
    float pose[12];       /* object -> camera [R|t], mm, row-major binary32 */
} perch_placed;

/* The edges from one state (n_state placed objects, host array, in placement
 * order) to object mesh_id (label) at each of n candidate poses:
 *   poses_dev:  n*12 binary32 (device)
 *   valid_dev:  n int32, 1 when the successor is monotone (device, written)
 *   jr_dev, jo_dev: n int32 edge costs, 0 for a successor that is not
 *               monotone (device, written)
 *   nr_dev, nq_dev: n int32 |dR \ C| and the observed points charged, or
 *               NULL (device, written)
 * The state's planes are composed on hip_stream at each call; with
 * n_state > 0 the call blocks until the composition has checked that the
 * state is monotone itself (PERCH_EINVAL when not), then scores
 * asynchronously. */
perch_status perch_msg_expand(perch_ctx *ctx, int32_t scene_id, const perch_placed *state, int32_t n_state,
                              int32_t mesh_id, int32_t label, const float *poses_dev, int32_t n,
                              int32_t *valid_dev, int32_t *jr_dev, int32_t *jo_dev, int32_t *nr_dev,
                              int32_t *nq_dev, void *hip_stream);

/* One object of a tree search: its mesh, label and n_poses candidate poses
 * (n_poses*12 binary32, device). */
typedef struct {
    int32_t mesh_id, label, n_poses;
    const float *poses_dev;
} perch_msg_object;

/* Beam search over the tree of n_obj objects (1..32).  Level by level it
 * keeps the `beam` states of least (cost, sequence) -- a state's cost is
 * the sum of its edge costs, sequences compare lexicographically as
 * (object index, pose index) pairs -- and scores every successor of each
 * on the GPU; beam 0 keeps every state (an exhaustive search, refused with
 * PERCH_ENOMEM when a level's states do not fit the HBM budget).  Returns
 * the goal of least (cost, sequence):
 *   order_host[l], pose_host[l]: n_obj int32 each, the object placed at
 *               level l and its pose index (-1 when no monotone goal exists)
 *   cost_host:  its cost (-1 when none)
 *   scored_host: successors scored, or NULL
 * Synchronous. */
perch_status perch_msg_search(perch_ctx *ctx, int32_t scene_id, const perch_msg_object *objects, int32_t n_obj,
                              int32_t beam, int32_t *order_host, int32_t *pose_host, int64_t *cost_host,
                              int64_t *scored_host, void *hip_stream);

/* Kernel timing.  perch_profile_enable(ctx, 1) clears the record and from
 * then on brackets every kernel launch of the context with HIP events on the
 * launch stream; 0 stops recording.  perch_profile_read waits for the
 * recorded events and returns, per slot, the summed duration in
 * milliseconds and the number of launches since the last enable.  Slots:
 * 0 pose set-up/classification; scoring kernels by footprint class:
 * 1 tile and keys in LDS (256 or 512 threads), 2 tile and keys in LDS (1024
 * threads), 3 tile in LDS and keys in device memory, 4 tile and keys in
 * device memory; 5 argmin, 6 scene preparation, 7 render (and kNN I's rasterization),
 * 8 ICP refinement, 9 tree successors, 10 kNN I distances and reductions,
 * 11 a prepared batch's whole graph replay (perch_batch_launch: descriptor
 * upload, set-up, the four scoring classes, argmin, result download; the
 * kernels inside a graph are not bracketed one by one). */
perch_status perch_profile_enable(perch_ctx *ctx, int32_t enable);
perch_status perch_profile_read(perch_ctx *ctx, int32_t n_slots, double *total_ms, int32_t *launches);

/* Footprint class (0..3, the scoring slots 1..4 of the profiler) that the
 * last perch_score_poses call on hip_stream assigned to each of its n poses:
 * class_host[i] for pose i.  Blocks until that call has finished.  Meant for
 * inspection and work accounting. */
perch_status perch_last_classes(perch_ctx *ctx, void *hip_stream, int32_t n, int32_t *class_host);

/* Launch tuning: how the poses of a launch are spread over the scoring
 * kernels.  No setting changes any result, only which work-group scores
 * which pose and in what order.
 *   small_block:  threads per work-group of the smallest LDS class, 256 or
 *                 512 (0 = 512); such work-groups get a quarter or a half of
 *                 a compute unit's LDS.
 *   small_words:  poses whose raster tile plus J_o key region needs at most
 *                 this many LDS words go to that class (0 = all that fit).
 *   grid[c]:      persistent work-groups of footprint class c (0 = as many
 *                 as are resident at once on the device).
 *   order:        1 = each class scores its poses in set-up order; 2 = by
 *                 image strip (one per XCD, each work-group starting on its
 *                 own XCD's strip), then costliest first -- or, in launches
 *                 over several scenes, scene by scene (0 = 2).
 *   key_bands:    for poses whose J_o keys do not fit in LDS beside the
 *                 raster tile: 1 = keys in device memory, 2 = keys in LDS,
 *                 one band of rows at a time (0 = 2).
 * The setting applies to launches enqueued afterwards, and to batches
 * created afterwards (a batch keeps the setting it was created with).
 * NULL restores the defaults.  perch_get_tuning returns the values in force,
 * defaults resolved. */
typedef struct {
    int32_t small_block;
    int32_t small_words;
    int32_t grid[4];
    int32_t order;
    int32_t key_bands;
} perch_tuning;
perch_status perch_set_tuning(perch_ctx *ctx, const perch_tuning *tuning);
perch_status perch_get_tuning(perch_ctx *ctx, perch_tuning *out);

/* Message describing the last error on the calling thread ("" if none). */
const char *perch_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PERCH_H */
