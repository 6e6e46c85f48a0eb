// Internal interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace perch {

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
constexpr int kBlockPx = 8;         // side of the depth-range blocks (pixels)
constexpr int kMaxTris = 65535;     // triangle index lives in 16 bits of the key
constexpr int kNumClasses = 3;      // LDS small, LDS large, global overflow

// Per-pose screen regions, computed by the setup kernel.
struct PoseInfo {
    int tx0, ty0, tw, th;   // raster tile (clipped to the image), may be empty
    int vx0, vy0, vw, vh;   // region holding every observed pixel that may lie in V(O)
};

struct SceneDev {
    const uint16_t *depth;   // H*W mm
    const int2 *oxy;         // H*W (Xq, Yq) in 1/16 mm
    const float4 *olab;      // H*W CIELAB (RGB scenes) or null
    const int32_t *labels;   // H*W or null
    const uint32_t *oblk;    // bw*bh: min depth | max depth << 16 of valid pixels
    const double *kx;        // W: 16 (i - cx) / fx
    const double *ky;        // H: 16 (j - cy) / fy
    const int2 *thdr;        // H*W nearest-neighbour table header: {first entry, lo | n << 16}
    const int32_t *tnn;      // entry (pixel, lo + e): nearest observed pixel within delta, -1 none
    int W, H, bw, bh;
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

struct Work {
    const float *poses;      // n * 12
    int n;
    int label;
    int32_t *jr, *jo, *nr, *nq;
    PoseInfo *info;          // n
    int *lists;              // kNumClasses * n pose indices
    int *counts;             // kNumClasses counters
    uint32_t *gscratch;      // overflow tiles
    size_t gscratch_stride;  // uint32 words per overflow slot
    int cap_small, cap_large;
    int vbox_label[4];       // label mode: x0, y0, w, h of the label's pixels
};

// Launch configuration chosen by the runtime (and the tuner).
struct LaunchCfg {
    int cap_small;      // LDS tile capacity (pixels), class 0
    int cap_large;      // class 1
    int grid_small, grid_large, grid_ovf;
};

// Upper bound on the 8x8 blocks of any tile of at most `cap` pixels inside a
// W x H image: ceil(w/8) ceil(h/8) <= cap/64 + 7 (W + H)/64 + 1.
inline int nbcap_for(int cap, int W, int H) { return cap / 64 + (W + H) / 4 + 4; }
size_t lds_bytes_for(int cap, int W, int H, int wtx, int wty);
hipError_t upload_colour_table(const float *lin256);

hipError_t launch_scene_prep(const SceneDev &s, const uint8_t *rgb_dev, int2 *oxy, float4 *olab,
                             uint32_t *oblk, hipStream_t st);
// Nearest-neighbour table of the observed cloud: per pixel the depth range
// that can have an observed point within delta, then one entry per depth.
hipError_t launch_table_ranges(const SceneDev &s, uint32_t *tmp, int2 *thdr, long long *total, hipStream_t st);
hipError_t launch_table_fill(const SceneDev &s, int32_t *tnn, hipStream_t st);
// Words of the LDS "explained" bitmap for a tile of at most `cap` pixels.
inline int bmcap_for(int cap, int W, int H, int wtx, int wty)
{
    const long long bits = (long long)cap + 2LL * wtx * H + 2LL * wty * W + 4LL * wtx * wty;
    return (int)(bits / 32 + 2);
}
hipError_t launch_setup(const SceneDev &s, const MeshDev &m, const Work &w, hipStream_t st);
hipError_t launch_score_class(const SceneDev &s, const MeshDev &m, const Work &w, const LaunchCfg &c, int cls,
                              hipStream_t st);

// Kernel slots reported by the profiler (perch_profile_read).
enum ProfSlot { kProfSetup = 0, kProfSmall = 1, kProfLarge = 2, kProfOverflow = 3, kProfArgmin = 4,
                kProfScenePrep = 5, kProfRender = 6, kNumProfSlots = 8 };
hipError_t launch_render(const SceneDev &s, const MeshDev &m, const float *poses, int n,
                         uint32_t *keys, uint16_t *depth, uint8_t *rgb, int32_t *tri,
                         hipStream_t st);
hipError_t launch_argmin(const int32_t *jr, const int32_t *jo, int n, int32_t *out2,
                         hipStream_t st);

}  // namespace perch
