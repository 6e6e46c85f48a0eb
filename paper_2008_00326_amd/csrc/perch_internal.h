// Internal interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace perch {

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
constexpr int kMaxTris = 65535;     // triangle index lives in 16 bits of the key
constexpr int kNoPoint = -(1 << 28); // Zq of a pixel without a depth reading: never within delta
constexpr int kNumClasses = 4;      // LDS small, LDS large, LDS tile + device keys, device memory
constexpr int kNumBuckets = 16;     // cost buckets of the per-class work order
constexpr int kNumStrips = 8;       // image strips of the work order, one per XCD
constexpr int kNumSegs = kNumClasses * kNumStrips;
constexpr int kNumOrders = kNumSegs * kNumBuckets;
// Launch counters (ints): per-class pose counts; per-(class, strip) work
// cursors, segment starts and lengths in the class list; per-(class,
// strip, bucket) counts and fill cursors of the ordered lists.
constexpr int kCntClass = 0;
constexpr int kCntNext = kCntClass + kNumClasses;
constexpr int kCntSegStart = kCntNext + kNumSegs;
constexpr int kCntSegLen = kCntSegStart + kNumSegs;
constexpr int kCntBucket = kCntSegLen + kNumSegs;
constexpr int kCntFill = kCntBucket + kNumOrders;
constexpr int kCounterInts = kCntFill + kNumOrders;

// Per-pose screen regions, computed by the setup kernel.
struct PoseInfo {
    int tx0, ty0, tw, th;   // raster tile (clipped to the image), may be empty
    int vx0, vy0, vw, vh;   // region holding every observed pixel that may lie in V(O)
    int jx0, jy0, jw, jh;   // part of the V region within reach of a rendered point
    int item, local;        // work item and pose index within it
    int order;              // (class * kNumStrips + strip) * kNumBuckets + sub-key (cost or scene group)
};

struct SceneDev {
    const uint16_t *depth;   // H*W mm
    const int4 *opt;         // H*W (Xq, Yq, Zq, 0) in 1/16 mm; Zq = kNoPoint without a reading
    const float4 *olab;      // H*W CIELAB (RGB scenes) or null
    const int32_t *labels;   // H*W or null
    const double *kx;        // W: 16 (i - cx) / fx
    const double *ky;        // H: 16 (j - cy) / fy
    const float *ax;         // W: f (delta + 1/4) sqrt(1 + ((i - cx) / fx)^2), rounded up
    const float *ay;         // H: the same for rows
    const int2 *thdr;        // H*W nearest-neighbour table header: {first entry, lo | n << 16} (null: hash)
    const int32_t *tnn;      // entry (pixel, lo + e): nearest observed pixel within delta, -1 none
    const int *hstart;       // voxel hash (hash scenes): 2^hbits + 1 bucket starts into hpts
    const int4 *hpts;        // observed points (Xq, Yq, Zq, pixel) grouped by bucket
    int hshift, hbits;       // cell edge 2^hshift (1/16 mm units, >= dq); 2^hbits buckets
    int W, H;
    int wtx, wty;            // window half-sizes that contain every neighbour pair of the scene
    float fx, fy, cx, cy;
    int dq, dq2, dzmm;       // delta in 1/16 mm, its square, floor(dq / 16)
    float delta, tau;
    uint32_t flags;
    int stride;
};

struct MeshDev {
    const float4 *verts;     // xyz, w unused
    const int4 *tris;        // vertex indices, w unused
    const uint32_t *vrgb;    // packed sRGB8 (r | g << 8 | b << 16) or null
    int nv, nt;
    float lo[3], hi[3];      // object-frame AABB
};

// One (scene, object, candidate poses) slice of a launch.
struct ItemDev {
    int scene, mesh;         // indices into the launch's scene and mesh tables
    int label, n;            // object label; number of poses
    int first;               // global index of the item's first pose in the launch
    int key32;               // 32-bit LDS keys are exact for this scene
    int vbox[4];             // label mode: x0, y0, w, h of the label's pixels
    const float *poses;      // n * 12
    int32_t *jr, *jo, *nr, *nq;
    uint8_t *rflag, *oflag;  // per pose a W*H image of each pixel's class (inspection), or null
};

struct LaunchHdr {
    int n_items, n_poses, n_scenes;
};

// Device-resident descriptors of one launch (header, items, scenes and
// meshes live contiguously in device memory) and its work buffers.
struct Work {
    const LaunchHdr *hdr;
    const ItemDev *items;    // sorted by `first`
    const SceneDev *scenes;
    const MeshDev *meshes;
    int cap_poses;           // capacity of info and each class list
    PoseInfo *info;          // cap_poses
    int *lists;              // kNumClasses * cap_poses global pose indices
    int *counts;             // kCounterInts launch counters (layout above)
    int sort;                // order each class list by image strip, then costliest first
    int key_bands;           // J_o regions too large for LDS are keyed in bands of rows (class 1)
    uint32_t *gscratch;      // device-memory slots of classes 2 (keys) and 3 (tile + keys)
    size_t slot_base[kNumClasses];   // first word of each class's slots
    size_t slot_words[kNumClasses];  // words per work-group slot
    size_t dev_tile_words;   // class 3: words of the slot's tile (keys follow)
    int cap_small, cap_large; // LDS words (tile + keys) of the two LDS classes
    float4 *lab;             // RGB: CIELAB of each inlier, one slot of tile pixels per work-group, or null
    size_t lab_base[kNumClasses];    // first entry of each class's slots
    size_t lab_px[kNumClasses];      // entries per work-group slot (the class's largest tile)
    int32_t *best;           // n_items x {index, J} of the per-item minimum, or null
};

// Launch configuration chosen by the runtime (and the tuner).
struct LaunchCfg {
    int small_block;    // threads per work-group of class 0 (256 or 512)
    int cap_small;      // LDS words per work-group (tile + keys), class 0
    int cap_large;      // classes 1 and 2 (class 2: tile only)
    int grid[kNumClasses];
    int sort;           // cost-ordered class lists
    int key_bands;      // banded J_o keys in LDS instead of device-memory keys
};

hipError_t upload_colour_table(const float *lin256);
// Allow each scoring kernel all the LDS a work-group can hold beside its
// static LDS (once per device); static_bytes receives the static LDS of the
// 256-, 512- and 1024-thread kernels (the largest over their variants).
hipError_t prepare_score_kernels(int lds_per_group, int static_bytes[3]);

hipError_t launch_scene_prep(const SceneDev &s, const uint8_t *rgb_dev, int4 *opt, float4 *olab, hipStream_t st);
// Nearest-neighbour table of the observed cloud: per pixel the depth range
// that can have an observed point within delta, then one entry per depth.
hipError_t launch_table_ranges(const SceneDev &s, uint32_t *tmp, int2 *thdr, long long *total, long long *blk,
                               hipStream_t st);
// Block sums the table scan needs (long long each).
int table_scan_blocks(int n_pixels);
// Fills the table; entries at or past `cap` are not written (a table sized
// on the host holds exactly the count the ranges kernels reach).
hipError_t launch_table_fill(const SceneDev &s, int32_t *tnn, long long cap, hipStream_t st);
constexpr uint32_t kHashFlag = 1u << 9;   // PERCH_HASH
// Uniform-grid voxel hash of the observed cloud: count points per bucket,
// exclusive scan into s.hstart (2^hbits + 1 ints), scatter into s.hpts.
// count: 2^hbits ints of work space; blk: table_scan_blocks(2^hbits) long longs.
hipError_t launch_hash_build(const SceneDev &s, int *count, long long *blk, hipStream_t st);
// A launch: zero the counters, classify every pose (grid sized for
// `poses_grid` poses; the kernels read the real count from the header) and,
// with w.sort, order each class list by cost bucket; run the four scoring
// classes, then the per-item argmin if w.best is set.
hipError_t launch_setup(const Work &w, int poses_grid, hipStream_t st);
hipError_t launch_score_class(const Work &w, const LaunchCfg &c, int cls, bool any_rgb, bool any_pv, hipStream_t st);
hipError_t launch_item_argmin(const Work &w, int items_grid, hipStream_t st);
// Descriptor block of a launch written by a kernel that takes the bytes by
// value (no host staging); at most kDescArgBytes bytes.
constexpr int kDescArgBytes = 512;
hipError_t launch_desc_write(const void *bytes, size_t n, void *dst, hipStream_t st);

// ICP refinement of candidate poses: arguments of one launch.
struct IcpArgs {
    SceneDev s;
    MeshDev m;
    const float *poses;      // n * 12
    int n, label;
    int iterations, stride, dof, min_points;
    int method;              // 0 point-to-point, 1 plane-to-plane GICP (6-DoF)
    int rq, rq2;             // correspondence radius in 1/16 mm and its square
    int box[4];              // x0, y0, x1, y1 (inclusive) holding every target pixel (label volumes:
                             // the label's pixels; x1 < x0 when there are none)
    float *refined;          // n * 12
    int32_t *iters, *matched; // or null
    int lds_words;           // dynamic LDS per work-group: the tile when it fits, then projected vertices
    uint32_t *tiles;         // per work-group: W*H tile words (tiles larger than the LDS)
    int4 *pts;               // per work-group: pts_cap source points, pts_cap mapped points (w: the match),
                             // and for GICP pts_cap source normals
    size_t pts_cap;
    int *cursor;             // pose cursor, zeroed by the launch
};
hipError_t launch_icp(const IcpArgs &a, int grid, hipStream_t st);
// Allow the ICP kernel all the LDS a work-group can hold beside its static
// LDS (once per device); *lds_words receives that dynamic capacity.
hipError_t prepare_icp_kernel(int lds_per_group, int *lds_words);

// 6-DoF pose proposals of one object: viewpoint x in-plane angle x depth.
struct ProposalArgs {
    int M, N, T, n;
    double zmin, zmax, step;   // depth of proposal t: zmin + t * step
    double uc, vc;             // the label box centre (pixels)
    double centre[3];          // object-frame centre of the mesh's AABB
    float fx, fy, cx, cy;
    float *out;                // n * 12
};
hipError_t launch_proposals(const ProposalArgs &a, hipStream_t st);

// Monotone Scene Generation tree: the full-image planes of one state.
struct MsgState {
    uint16_t *depth;          // composed depth in mm, 0 where no placed object draws
    uint16_t *pts;            // depth where the pixel is a point of the composed R \ C, else 0
    uint32_t *rgb;            // packed sRGB8 of the composed render (RGB scenes), else null
    uint8_t *cov;             // 1 where the observed point lies in a placed object's volume
    unsigned long long *near; // per observed pixel: min (d2 << 32 | pixel) over R \ C within delta, ~0 none
};
// Bytes of the planes of one state of n pixels, each plane 256-byte aligned.
inline size_t msg_state_bytes(size_t n)
{
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return up(2 * n) + up(2 * n) + up(4 * n) + up(n) + up(8 * n);
}
inline MsgState msg_state_at(void *base, size_t n, bool rgb)
{
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = (char *)base;
    MsgState st;
    st.depth = (uint16_t *)p;
    p += up(2 * n);
    st.pts = (uint16_t *)p;
    p += up(2 * n);
    st.rgb = rgb ? (uint32_t *)p : nullptr;
    p += up(4 * n);
    st.cov = (uint8_t *)p;
    p += up(n);
    st.near = (unsigned long long *)p;
    return st;
}
// Append one object (mesh m at pose P) to a state in place.
struct MsgAddArgs {
    SceneDev s;
    MeshDev m;
    const float *pose;        // 12 binary32 (device)
    int label;
    MsgState st;
    uint32_t *keys;           // W*H raster keys
    int *flag;                // set to 1 when the object occludes the state (not monotone)
};
// Score every successor of one state: one object at each of n poses.
struct MsgArgs {
    SceneDev s;
    MeshDev m;
    const float *poses;       // n * 12
    int n, label;
    int vbox[4];              // label volumes: x0, y0, w, h of the label's pixels
    MsgState st;
    int32_t *valid, *jr, *jo, *nr, *nq;   // nr, nq may be null
    int lds_words;            // dynamic LDS per work-group: the tile when it fits, then projected vertices
    uint32_t *tiles;          // per work-group: W*H tile words (tiles larger than the LDS)
    int *cursor;              // pose cursor, zeroed by the launch
};
hipError_t upload_msg_colour_table(const float *lin256);
hipError_t msg_state_clear(const SceneDev &s, const MsgState &st, hipStream_t stream);
hipError_t msg_state_add(const MsgAddArgs &a, hipStream_t stream);
// The per-observed-pixel nearest state point, after the last msg_state_add.
hipError_t msg_state_near(const SceneDev &s, const MsgState &st, hipStream_t stream);
hipError_t launch_msg(const MsgArgs &a, int grid, hipStream_t stream);
hipError_t prepare_msg_kernel(int lds_per_group, int *lds_words);

// kNN I (the paper's fully parallel neighbour search): one pose at a time,
// with every (rendered, observed) distance in a two-dimensional array.
struct Knn1Args {
    SceneDev s;
    MeshDev m;
    const float *poses;       // n * 12
    int label;
    uint32_t *keys;           // W*H raster keys
    int4 *pts;                // R \ C: (X, Y, Z, pixel), at most W*H
    uint32_t *pcol;           // W*H packed sRGB8 of the rendered points (RGB scenes)
    const int *obs;           // n_obs pixels with a reading
    int n_obs;
    uint32_t *dist;           // L * n_obs squared distances (saturated)
    uint8_t *marked;          // W*H marks of nearest-neighbour J_o, or null
    int *counts;              // L, J_r, J_o, Q of the current pose
    int32_t *jr, *jo, *nr, *nq;
};
hipError_t upload_knn1_colour_table(const float *lin256);
hipError_t knn1_observed(const SceneDev &s, int *obs, int *n_obs, hipStream_t st);
// Render pose p and list its R \ C points (count in counts[0]).
hipError_t knn1_render(const Knn1Args &a, int p, hipStream_t st);
// Distances, rows and columns of pose p with L rendered points; writes its outputs.
hipError_t knn1_score(const Knn1Args &a, int p, int L, hipStream_t st);

// Kernel slots reported by the profiler (perch_profile_read).
enum ProfSlot { kProfSetup = 0, kProfClass0 = 1, kProfArgmin = 5, kProfScenePrep = 6, kProfRender = 7,
                kProfIcp = 8, kProfMsg = 9, kProfKnn1 = 10, kProfGraph = 11, kNumProfSlots = 12 };
hipError_t launch_render(const SceneDev &s, const MeshDev &m, const float *poses, int n,
                         uint32_t *keys, uint16_t *depth, uint8_t *rgb, int32_t *tri,
                         hipStream_t st);


}  // namespace perch
