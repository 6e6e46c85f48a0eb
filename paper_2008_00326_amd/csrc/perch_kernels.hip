// gfx950 kernels for PERCH 2.0 pose scoring.
//
// Per candidate pose (Sec. IV-A "Parallel Rendering" / "Parallel Cost
// Computation", Eq. 1-4), one work-group:
//   1. rasterize the mesh into a tile of 32-bit keys (depth mm << 16 |
//      triangle index) in LDS, min-combined with ds_min_u32;
//   2. resolve: drop occluders (Eq. 3, C from the observed depth) and pixels
//      off the downsampling grid;
//   3. J_r: each rendered point's nearest observed point within delta is one
//      lookup in the scene's nearest-neighbour table; every inlier then
//      marks the observed points within delta of it with its (squared
//      distance, index) key, one wave per inlier;
//   4. J_o: an observed point inside V(O) is explained iff it was marked, and
//      its key names its nearest rendered point;
//   5. RGB mode: CIEDE2000 of each point against its nearest neighbour
//      (Eq. 4), in binary32, over dense queues;
//   6. wave ballot + popcount of the outlier predicates.
// Geometry and depth use integer / binary64 arithmetic that the oracle
// reproduces exactly (no FMA contraction: built with -ffp-contract=off).

#include "perch_device.h"

#include <math.h>
#include <string.h>

namespace perch {

// ------------------------------------------------------------------ search

// ceil(2^16 / w) for w = 1..64: q / w = (q * c_rcp16[w]) >> 16 exactly for
// q < 256 (the error term q (c - 2^16 / w) / 2^16 stays below 1 / w).
__constant__ uint32_t c_rcp16[65] = {
    0,    65536, 32768, 21846, 16384, 13108, 10923, 9363, 8192, 7282, 6554, 5958, 5462, 5042, 4682, 4370, 4096,
    3856, 3641,  3450,  3277,  3121,  2979,  2850,  2731, 2622, 2521, 2428, 2341, 2260, 2185, 2115, 2048, 1986,
    1928, 1873,  1821,  1772,  1725,  1681,  1639,  1599, 1561, 1525, 1490, 1457, 1425, 1395, 1366, 1338, 1311,
    1286, 1261,  1237,  1214,  1192,  1171,  1150,  1130, 1111, 1093, 1075, 1058, 1041, 1024};

// Nearest-neighbour keys of the J_o region: smallest (squared distance,
// tile index of the rendered point) over the rendered points within delta.
// 32 bits (distance << 16 | index) in LDS, 64 bits in device memory.
template <bool G> struct KeyOf;
template <> struct KeyOf<false> {
    using T = uint32_t;
    static constexpr T kEmpty = 0xFFFFFFFFu;
    __device__ static T make(int d2, int k) { return ((uint32_t)d2 << 16) | (uint32_t)k; }
    __device__ static int index(T key) { return (int)(key & 0xFFFFu); }
    __device__ static void min(T *p, T v) { atomicMin(p, v); }
    __device__ static T load(const T *p) { return *p; }
    __device__ static void store(T *p, T v) { *p = v; }
};
template <> struct KeyOf<true> {
    using T = unsigned long long;
    static constexpr T kEmpty = ~0ULL;
    __device__ static T make(int d2, int k) { return ((unsigned long long)(uint32_t)d2 << 32) | (uint32_t)k; }
    __device__ static int index(T key) { return (int)(key & 0xFFFFFFFFu); }
    __device__ static void min(T *p, T v) { __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ static T load(const T *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ static void store(T *p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
};

// Key update of an observed point q by rendered point (X, Y, Z) with tile
// index k, if the two lie within delta.  The three offsets saturate to 16
// bits (v_cvt_pk_i16_i32) and two v_dot2_i32_i16 sum their squares: at most
// 3 * 2^30 < 2^32, so the sum read unsigned is exact when no offset
// saturated and exceeds dq^2 (dq < 2^13) when one did.
typedef short perch_s2 __attribute__((ext_vector_type(2)));
template <bool G>
__device__ __forceinline__ void mark_one(int3 q, int X, int Y, int Z, int k, int dq2, typename KeyOf<G>::T *key)
{
    using K = KeyOf<G>;
    const perch_s2 xy = __builtin_amdgcn_cvt_pk_i16(q.x - X, q.y - Y);
    const perch_s2 z0 = __builtin_amdgcn_cvt_pk_i16(q.z - Z, 0);
    const uint32_t d2 = (uint32_t)__builtin_amdgcn_sdot2(xy, xy, __builtin_amdgcn_sdot2(z0, z0, 0, false), false);
    if (d2 <= (uint32_t)dq2) K::min(key, K::make((int)d2, k));
}

// Per-inlier marking parameters, computed once by the thread that queues
// the inlier: its point (X, Y) in 1/16 mm and its window half-sizes.
__device__ __forceinline__ void mark_params(const SceneDev &s, int i, int j, int d, int *X, int *Y, int *wuv)
{
    *X = (int)rint(gld(s.kx + i) * (double)d);
    *Y = (int)rint(gld(s.ky + j) * (double)d);
    const float iz = window_inv(d, s.delta + 0.25f);
    *wuv = window_half(gld(s.ax + i), iz, s.W) | (window_half(gld(s.ay + j), iz, s.H) << 16);
}

// Squared pixel radius of the ellipse that holds every observed neighbour
// of rendered point r = (i, j, d), in column units: an observed point within
// delta of r sits at column and row offsets (di, dj) with
// di^2 + (fx/fy)^2 dj^2 <= fx^2 (1 + xh^2 + yh^2) e^2 / (d - e)^2, where
// e = delta + 1/4 mm (the 1/16 mm rounding of both points inside it) and
// (xh, yh) = ((i - cx)/fx, (j - cy)/fy).  With o - r = v, |v| <= e, the
// column offset is fx (v_x - xh v_z) / (d + v_z): the numerators of both
// offsets are M v with M = [1 0 -xh; 0 1 -yh], whose largest singular value
// is sqrt(1 + xh^2 + yh^2), and d + v_z >= d - e.  The binary32 value is
// raised by 1e-5 relative, above its rounding; infinity when d - e <= 1 mm,
// where no bound is taken.
__device__ __forceinline__ float mark_ellipse(const SceneDev &s, int i, int j, int d)
{
    const float e = s.delta + 0.25f;
    const float den = (float)d - e;
    if (!(den > 1.0f)) return INFINITY;
    const float xh = ((float)i - s.cx) / s.fx, yh = ((float)j - s.cy) / s.fy;
    const float r = s.fx * e / den;
    return r * r * (1.0f + xh * xh + yh * yh) * 1.00001f;
}

// Scene values the marking loop reads, held in scalar registers for a pose.
struct MarkScene {
    const int4 *opt;
    int W, H, dq2;
};

template <class T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    const unsigned long long v = (unsigned long long)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ MarkScene mark_scene(const SceneDev &s)
{
    MarkScene m;
    m.opt = uniform_ptr(s.opt);
    m.W = __builtin_amdgcn_readfirstlane(s.W);
    m.H = __builtin_amdgcn_readfirstlane(s.H);
    m.dq2 = __builtin_amdgcn_readfirstlane(s.dq2);
    return m;
}

// The whole wave takes one rendered inlier r = (i, j, d), tile index k, and
// visits every observed pixel of r's window inside the J_o region: each
// observed point within delta of r min-combines (d2, k) into its key.  This
// marks the points that r explains (Eq. 3) and, over all r, leaves each
// observed point's nearest rendered neighbour (Eq. 4).  A window of at most
// 256 pixels goes in at most four row-major rounds of 64, every load issued
// first; a larger one no wider than a wave in whole rows per round (64 /
// width rows, a lane keeps its column and steps its row by a constant),
// four rounds per iteration; a wider one in row-major order, four pixels
// per lane per round.  Image and key offsets are 32-bit, products 24-bit
// (every index here is below 2^24).
template <bool G>
__device__ void wave_mark(const MarkScene &s, int i, int j, int d, int k, int X, int Y, int wuv,
                          typename KeyOf<G>::T *keys, int jx0, int jy0, int jw, int jh, int lane)
{
    const int wu = wuv & 0xFFFF, wv = wuv >> 16;
    const int i0 = max(max(i - wu, 0), jx0), i1 = min(min(i + wu, s.W - 1), jx0 + jw - 1);
    const int j0 = max(max(j - wv, 0), jy0), j1 = min(min(j + wv, s.H - 1), jy0 + jh - 1);
    if (i0 > i1 || j0 > j1) return;
    const int ww = i1 - i0 + 1, wh = j1 - j0 + 1;
    const int Z = 16 * d;
    const int dq2 = s.dq2;
    const int ws = ww * wh;
    const int W = s.W;
    const int pbase = j0 * W + i0;                     // window origin in the image
    const int kbase = (j0 - jy0) * jw + (i0 - jx0);    // and among the keys
    if (ws <= 256 && ww <= 64) {
        // the whole window in at most four row-major rounds of 64 pixels,
        // every load issued first (lanes past the window's end load its last
        // pixel and mark nothing); (q * ceil(2^16 / ww)) >> 16 is q / ww
        // exactly for q < 256
        const uint32_t rc = c_rcp16[ww];
        const int4 *wopt = s.opt + pbase;
        typename KeyOf<G>::T *wkey = keys + kbase;
        int3 q[4];
        int kk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (64 * u < ws) {
                const int f = min(64 * u + lane, ws - 1);
                const int fy = (int)(__umul24((uint32_t)f, rc) >> 16), fx = __mul24(fy, -ww) + f;
                kk[u] = __mul24(fy, jw) + fx;
                q[u] = opt_at(wopt, (uint32_t)(__mul24(fy, W) + fx));
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (64 * u + lane < ws) mark_one<G>(q[u], X, Y, Z, k, dq2, wkey + kk[u]);
        return;
    }
    if (ww <= 64) {
        const uint32_t rc = c_rcp16[ww];
        const int rows = (int)((64u * rc) >> 16);
        const int r = (int)(__umul24((uint32_t)lane, rc) >> 16), c = lane - __mul24(r, ww);
        if (r >= rows) return;
        const int step = __mul24(rows, W), kstep = __mul24(rows, jw);
        int pix = pbase + __mul24(r, W) + c;
        int kk = kbase + __mul24(r, jw) + c;
        int row = r;
        for (; row + 3 * rows < wh; row += 4 * rows) {
            int3 q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = opt_at(s.opt, (uint32_t)(pix + u * step));
#pragma unroll
            for (int u = 0; u < 4; ++u) mark_one<G>(q[u], X, Y, Z, k, dq2, keys + kk + u * kstep);
            pix += 4 * step;
            kk += 4 * kstep;
        }
        int3 q[3];
#pragma unroll
        for (int u = 0; u < 3; ++u)
            q[u] = row + u * rows < wh ? opt_at(s.opt, (uint32_t)(pix + u * step)) : make_int3(0, 0, kNoPoint);
#pragma unroll
        for (int u = 0; u < 3; ++u)
            if (row + u * rows < wh) mark_one<G>(q[u], X, Y, Z, k, dq2, keys + kk + u * kstep);
        return;
    }
    const float inv = 1.0f / (float)ww;
    for (int q0 = 0; q0 < ws; q0 += 256) {
        int kk[4];
        int3 qv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + 64 * u + lane;
            const int qy = window_row(q, ww, inv), qx = q - qy * ww;
            kk[u] = kbase + qy * jw + qx;
            qv[u] = q < ws ? opt_at(s.opt, (uint32_t)(pbase + qy * W + qx)) : make_int3(0, 0, kNoPoint);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + 64 * u + lane < ws) mark_one<G>(qv[u], X, Y, Z, k, dq2, keys + kk[u]);
    }
}

// Wave-wide minimum and maximum of a lane value.
__device__ __forceinline__ int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Inliers a wave marks together, one per lane, at least: below it each
// inlier takes the whole wave (wave_mark), since the lanes' shared offset
// loop costs the same for few inliers as for 64.
constexpr int kLanesMin = 32;

// Marking of up to 64 inliers at once, one per lane (`act`): the wave steps
// through the union of the lanes' windows as offsets (dx, dy) from each
// lane's own pixel, four offsets per step with every load issued first, and
// a lane whose own window (clipped to the image and to the band
// [jx0, jx0 + jw) x [jy0, jy0 + jh)) holds the offset marks that observed
// pixel.  Each row of offsets is cut to the chord of the largest of the
// lanes' neighbour ellipses (E: mark_ellipse; c2 = (fx/fy)^2), which holds
// every lane's own.  Queued inliers come from neighbouring tile pixels, so
// one offset's loads and key updates fall on neighbouring pixels.  Offsets
// outside a lane's window re-read a pixel of it and mark nothing.
template <bool G>
__device__ void wave_mark_lanes(const MarkScene &s, bool act, int i, int j, int d, int k, int X, int Y, int wuv,
                                float E, float c2, typename KeyOf<G>::T *keys, int jx0, int jy0, int jw, int jh)
{
    const int wu = wuv & 0xFFFF, wv = wuv >> 16;
    int x0 = max(max(-wu, -i), jx0 - i), x1 = min(min(wu, s.W - 1 - i), jx0 + jw - 1 - i);
    int y0 = max(max(-wv, -j), jy0 - j), y1 = min(min(wv, s.H - 1 - j), jy0 + jh - 1 - j);
    const bool live = act && x0 <= x1 && y0 <= y1;
    const int DX0 = __builtin_amdgcn_readfirstlane(wave_min(live ? x0 : 1 << 20));
    const int DX1 = __builtin_amdgcn_readfirstlane(wave_max(live ? x1 : -(1 << 20)));
    const int DY0 = __builtin_amdgcn_readfirstlane(wave_min(live ? y0 : 1 << 20));
    const int DY1 = __builtin_amdgcn_readfirstlane(wave_max(live ? y1 : -(1 << 20)));
    if (DX0 > DX1) return;
    // non-negative binary32 values order as their bit patterns
    const float Em = __int_as_float(__builtin_amdgcn_readfirstlane(wave_max(live ? __float_as_int(E) : 0)));
    if (!live) x0 = x1 = y0 = y1 = 0;                 // idle lanes re-read their own pixel
    const int Z = 16 * d;
    const int dq2 = s.dq2;
    const int pix = live ? j * s.W + i : 0;
    const int kp = (j - jy0) * jw + (i - jx0);
    for (int dy = DY0; dy <= DY1; ++dy) {
        // the chord's half-width, rounded up past the binary32 error (the
        // row term lowered by 1e-5 relative, the root raised)
        const float t = Em - c2 * (float)(dy * dy) * 0.99999f;
        if (!(t >= 0.0f)) continue;
        const int hw = __builtin_amdgcn_readfirstlane((int)fminf(sqrtf(t) * 1.00001f, 65536.0f));
        const int rx0 = max(DX0, -hw), rx1 = min(DX1, hw);
        const int cy = min(max(dy, y0), y1);
        const bool rowok = live && cy == dy;
        const int prow = pix + cy * s.W, krow = kp + cy * jw;
        for (int dx = rx0; dx <= rx1; dx += 4) {
            int3 qv[4];
            int cx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                cx[u] = min(max(dx + u, x0), x1);
                qv[u] = opt_at(s.opt, (uint32_t)(prow + cx[u]));
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (rowok && cx[u] == dx + u) mark_one<G>(qv[u], X, Y, Z, k, dq2, keys + krow + cx[u]);
        }
    }
}

// Nearest-neighbour marks of the J_o region (J_o by marking): one bit per
// pixel, set when the pixel's observed point is the nearest neighbour of a
// rendered inlier.  G: the bitmap lives in device memory.
template <bool G> struct Marks;
template <> struct Marks<false> {
    __device__ static void clear(uint32_t *w) { *w = 0u; }
    __device__ static void set(uint32_t *b, int k) { atomicOr(b + (k >> 5), 1u << (k & 31)); }
    __device__ static bool test(const uint32_t *b, int k) { return (b[k >> 5] >> (k & 31)) & 1u; }
};
template <> struct Marks<true> {
    __device__ static void clear(uint32_t *w) { __hip_atomic_store(w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
    __device__ static void set(uint32_t *b, int k)
    {
        __hip_atomic_fetch_or(b + (k >> 5), 1u << (k & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static bool test(const uint32_t *b, int k)
    {
        return (__hip_atomic_load(b + (k >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> (k & 31)) & 1u;
    }
};

// kNN II (Sec. IV-A, parallel cost computation): the nearest observed point
// of rendered point (X, Y, Z) found by one thread scanning the whole observed
// cloud, as the paper's reduced-parallelism search does.  Same result as the
// scene table: the smallest (d², pixel index) within delta, or -1.  The scan
// address is uniform, so the points come through the scalar cache.
__device__ __noinline__ int scan_nn(const SceneDev &s, int X, int Y, int Z)
{
    const int lim = s.dq + 1, dq2 = s.dq2;
    const int n = s.W * s.H;
    int best = dq2 + 1, nn = -1;
    int p = 0;
    for (; p + 4 <= n; p += 4) {
        int4 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = gld(s.opt + p + u);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int dx = clamp_i32(q[u].x - X, -lim, lim);
            const int dy = clamp_i32(q[u].y - Y, -lim, lim);
            const int dz = clamp_i32(q[u].z - Z, -lim, lim);
            const int d2 = __mul24(dx, dx) + __mul24(dy, dy) + __mul24(dz, dz);
            if (d2 < best) {
                best = d2;
                nn = p + u;
            }
        }
    }
    for (; p < n; ++p) {
        const int4 q = gld(s.opt + p);
        const int dx = clamp_i32(q.x - X, -lim, lim);
        const int dy = clamp_i32(q.y - Y, -lim, lim);
        const int dz = clamp_i32(q.z - Z, -lim, lim);
        const int d2 = __mul24(dx, dx) + __mul24(dy, dy) + __mul24(dz, dz);
        if (d2 < best) {
            best = d2;
            nn = p;
        }
    }
    return nn;
}

// Marks observed pixel nn (the nearest neighbour of a rendered inlier) in
// the bitmap of the J_o region; pixels outside the region lie outside V(O).
template <bool KG>
__device__ __forceinline__ void mark_nn(uint32_t *bits, int nn, int W, int jx0, int jy0, int jw, int jh)
{
    const int ny = nn / W;
    const int jx = nn - ny * W - jx0, jy = ny - jy0;
    if (jx >= 0 && jx < jw && jy >= 0 && jy < jh) Marks<KG>::set(bits, jy * jw + jx);
}

__device__ __forceinline__ int wave_popc(bool pred)
{
    return __popcll(__ballot(pred));
}

// Number of lanes below this one whose bit is set in mask m.
__device__ __forceinline__ int lane_rank(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Make the LDS writes of a wave visible to all its lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Row of tile index k in a tile tw pixels wide (inv = 1 / tw in binary32).
// An LDS tile holds fewer than 2^16 pixels: there (k + 1/2) / tw, whose
// fraction lies at least 1 / (2 tw) from an integer, is computed with a
// relative error below 2^-22 and truncates to the exact quotient.  A
// device-memory tile can be larger and divides.
template <bool G>
__device__ __forceinline__ int tile_row(int k, int tw, float inv)
{
    if constexpr (G) return k / tw;
    else return (int)(((float)k + 0.5f) * inv);
}

// ------------------------------------------------------------------ per pose

template <int BLOCK, bool G, bool KG, bool RGB, bool PV>
__device__ void score_pose(const Work &w, int p, uint32_t *tile, typename KeyOf<KG>::T *keys, float4 *labs, int *cnt,
                           int2 *wq)
{
    using K = KeyOf<KG>;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const PoseInfo in = w.info[p];
    const ItemDev &it = w.items[in.item];
    const SceneDev &s = w.scenes[it.scene];
    const MeshDev &m = w.meshes[it.mesh];
    const bool rgb = RGB && (s.flags & 1u) != 0;
    float P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = it.poses[12 * (size_t)in.local + k];
    const int tpx = in.tw * in.th;
    const int jpx = in.jw * in.jh;
    const float tinv = 1.0f / (float)max(in.tw, 1);
    const MarkScene ms = mark_scene(s);
    // class images of the inspection entry point: rendered pixels 1 inlier,
    // 2 no neighbour, 3 colour mismatch, 4 occluded; observed pixels of V(O)
    // 1 explained, 2 no neighbour, 3 colour mismatch
    uint8_t *const rf = it.rflag ? it.rflag + (size_t)in.local * s.W * s.H : nullptr;
    uint8_t *const of = it.oflag ? it.oflag + (size_t)in.local * s.W * s.H : nullptr;
    const bool mark = (s.flags & 2u) != 0;
    const bool label_mode = (s.flags & (3u << 4)) == (2u << 4);
    const bool cyl = (s.flags & (3u << 4)) == (1u << 4);
    // J_o by nearest-neighbour marking: a bitmap over the J_o region instead
    // of keys, set by the inliers (after their colour test), with no search
    // and no colour test of its own.  Its poses are never banded.
    const bool nnm = PV && (s.flags & 64u) != 0;
    const bool knn2 = PV && (s.flags & 128u) != 0;     // J_r neighbours by the kNN II scan
    const bool hsh = PV && (s.flags & kHashFlag) != 0; // J_r neighbours through the voxel hash
    uint32_t *bits = reinterpret_cast<uint32_t *>(keys);
    const bool ocol = rgb && !nnm;

    const int band0 = (!nnm && !G && !KG && BLOCK == 1024 && tpx + jpx > w.cap_large) ? (w.cap_large - tpx) : jpx;
    for (int k = tid; k < tpx; k += BLOCK) tst<G>(tile + k, kEmptyKey);
    if (tid < 4) cnt[tid] = 0;
    // 0. with LDS to spare beyond the tile (the J_o keys are cleared only
    //    after the raster), every vertex is projected once for the pose
    const int tile_q = (tpx + 3) & ~3;
    const int4 *vcache = nullptr;
    if (!G && tpx > 0 && 4 * m.nv <= (BLOCK == 1024 ? w.cap_large : w.cap_small) - tile_q) {
        int4 *vc = reinterpret_cast<int4 *>(tile + tile_q);
        for (int v = tid; v < m.nv; v += BLOCK) vc[v] = pack_vtx(project_vertex(P, gld(m.verts + v), s));
        vcache = vc;
    }
    __syncthreads();

    // 1. raster
    if (tpx > 0) {
        for (int t0 = 0; t0 < m.nt; t0 += BLOCK) {
            const int t = t0 + tid;
            if (t < m.nt) raster_triangle<G>(s, m, P, t, in.tx0, in.ty0, in.tw, in.th, tile, vcache);
        }
    }
    __syncthreads();
    if (nnm) {
        for (int k = tid; k < (jpx + 31) >> 5; k += BLOCK) Marks<KG>::clear(bits + k);
    } else {
        for (int k = tid; k < min(jpx, band0); k += BLOCK) K::store(keys + k, K::kEmpty);
    }

    // 2. resolve: occluders (Eq. 3) and the downsampling stride
    int cL = 0;
    {
        // tile pixel of index k (clamped into the tile): key and image position
        auto rpixel = [&](int k, uint32_t &key, int &i, int &j) {
            const int kc = min(k, tpx - 1);
            key = k < tpx ? tld<G>(tile + kc) : kEmptyKey;
            const int ty = tile_row<G>(kc, in.tw, tinv), tx = kc - __mul24(ty, in.tw);
            i = in.tx0 + tx;
            j = in.ty0 + ty;
        };
        auto resolve = [&](int k, uint32_t key, int i, int j, int dob) {
            bool keep = false;
            if (key != kEmptyKey) {
                const int d = (int)(key >> 16);
                keep = s.stride == 1 || ((i % s.stride == 0) && (j % s.stride == 0));
                if (keep && mark && dob > 0 && 16 * dob + s.dq < 16 * d) {
                    const int pix = j * s.W + i;
                    if (!(label_mode && s.labels) || s.labels[pix] != it.label) {
                        keep = false;
                        if (rf) rf[pix] = 4;
                    }
                }
                if (!keep) tst<G>(tile + k, kEmptyKey);
            }
            cL += wave_popc(keep);
        };
        // two chunks a turn, both observed depths loaded first (every lane
        // loads, at a clamped pixel)
        for (int k0 = 0; k0 < tpx; k0 += 2 * BLOCK) {
            const int kA = k0 + tid, kB = k0 + BLOCK + tid;
            uint32_t keyA, keyB;
            int iA, jA, iB, jB;
            rpixel(kA, keyA, iA, jA);
            rpixel(kB, keyB, iB, jB);
            const int dA = mark ? (int)gld(s.depth + (uint32_t)(jA * s.W + iA)) : 0;
            const int dB = mark ? (int)gld(s.depth + (uint32_t)(jB * s.W + iB)) : 0;
            resolve(kA, keyA, iA, jA, dA);
            if (k0 + BLOCK < tpx) resolve(kB, keyB, iB, jB, dB);
        }
    }
    __syncthreads();

    // J_o keys held at once: the whole J_o region, or, for a pose of the
    // 1024-thread LDS class whose region does not fit beside its tile, bands
    // of rows; phases 3 and 4 then run once per band, every inlier marking
    // the band's keys, and the J_r counts are taken in the first band.
    int hb = in.jh;
    if (!nnm && !G && !KG && BLOCK == 1024 && in.jw > 0 && tpx + jpx > w.cap_large) hb = (w.cap_large - tpx) / in.jw;
    const int nb = in.jh > 0 ? (in.jh + hb - 1) / hb : 1;
    int cR = 0, cQ = 0, cO = 0;
    const double dl = (double)s.delta;
    // Phases 3 and 4 run without work-group barriers: each wave takes
    // 64-pixel blocks in turn and appends its work (inliers to mark and to
    // colour-test, explained observed points to colour-test) to its own
    // queue `q` of 128 entries in LDS, flushed 64 at a time -- a colour
    // test per lane, marking one inlier at a time with the whole wave.
    int2 *const q = wq + wave * 128;
    for (int b = 0; b < nb; ++b) {
        const bool first = b == 0;
        const int by0 = in.jy0 + b * hb;
        const int bh = in.jh > 0 ? min(hb, in.jy0 + in.jh - by0) : 0;
        const int bpx = in.jw * bh;
        if (!first) {
            __syncthreads();
            for (int k = tid; k < bpx; k += BLOCK) K::store(keys + k, K::kEmpty);
            __syncthreads();
        }

        // 3. J_r: nearest observed neighbour from the scene table (or the
        //    kNN II scan).  Queued inliers are colour-tested (Eq. 4, first
        //    band) and mark the observed points they explain.
        auto flush_r = [&](int n) {
            wave_lds_sync();
            int kk = 0, nn = -1, ei = 0, ej = 0, ed = 0, tri = 0;
            if (lane < n) {
                const int2 e = q[lane];
                kk = e.x;
                nn = e.y;
                const uint32_t key = tld<G>(tile + kk);
                const int ty = tile_row<G>(kk, in.tw, tinv), tx = kk - __mul24(ty, in.tw);
                ei = in.tx0 + tx;
                ej = in.ty0 + ty;
                ed = (int)(key >> 16);
                tri = (int)(key & 0xFFFFu);
            }
            if (rgb && first) {
                bool out = false;
                if (lane < n) {
                    const float4 lr = srgb_to_lab(triangle_colour(s, m, P, tri, ei, ej));
                    if (labs) labs[kk] = lr;     // kept for the J_o test of the points this inlier keys
                    out = ciede2000(lr, gld(s.olab + nn)) > s.tau;
                    if (nnm && !out) mark_nn<KG>(bits, nn, s.W, in.jx0, in.jy0, in.jw, in.jh);
                    if (rf) rf[ej * s.W + ei] = out ? 3 : 1;
                }
                cR += wave_popc(out);
            }
            if (bpx > 0 && !nnm) {
                int X = 0, Y = 0, wuv = 0;
                if (lane < n) mark_params(s, ei, ej, ed, &X, &Y, &wuv);
                if (n >= kLanesMin) {
                    const float E = lane < n ? mark_ellipse(s, ei, ej, ed) : 0.0f;
                    const float c2 = (s.fx / s.fy) * (s.fx / s.fy);
                    wave_mark_lanes<KG>(ms, lane < n, ei, ej, ed, kk, X, Y, wuv, E, c2, keys, in.jx0, by0, in.jw, bh);
                } else {
                    for (int t = 0; t < n; ++t)
                        wave_mark<KG>(ms, __builtin_amdgcn_readlane(ei, t), __builtin_amdgcn_readlane(ej, t),
                                      __builtin_amdgcn_readlane(ed, t), __builtin_amdgcn_readlane(kk, t),
                                      __builtin_amdgcn_readlane(X, t), __builtin_amdgcn_readlane(Y, t),
                                      __builtin_amdgcn_readlane(wuv, t), keys, in.jx0, by0, in.jw, bh, lane);
                }
            }
        };
        int qc = 0;
        // the queue step of one tile pixel: misses counted, flags, the
        // inliers queued (whole wave)
        auto rstep = [&](bool keyed, int k, int pix, int nn) {
            bool miss = false, need = false;
            if (keyed) {
                miss = first && nn < 0;
                if (rf && first && (nn < 0 || !rgb)) rf[pix] = nn < 0 ? 2 : 1;
                if (nnm && !rgb && nn >= 0) mark_nn<KG>(bits, nn, s.W, in.jx0, in.jy0, in.jw, in.jh);
                need = nn >= 0 && ((rgb && first) || (bpx > 0 && !nnm));
            }
            cR += wave_popc(miss);
            const unsigned long long mq = __ballot(need);
            if (need) q[qc + lane_rank(mq)] = make_int2(k, nn);
            qc += __popcll(mq);
            if (qc >= 64) {
                flush_r(64);
                wave_lds_sync();
                if (64 + lane < qc) q[lane] = q[64 + lane];     // the overflow moves to the front
                qc -= 64;
            }
        };
        // tile pixel of index k (clamped into the tile): key and image pixel
        auto tpixel = [&](int k, uint32_t &key, int &pix) {
            const int kc = min(k, tpx - 1);
            key = k < tpx ? tld<G>(tile + kc) : kEmptyKey;
            const int ty = tile_row<G>(kc, in.tw, tinv), tx = kc - __mul24(ty, in.tw);
            pix = (in.ty0 + ty) * s.W + in.tx0 + tx;
        };
        // four chunks a turn: every chunk's table entries are loaded before
        // any is queued
        for (int k0 = wave * 64; k0 < tpx; k0 += 4 * BLOCK) {
            uint32_t key[4];
            int pp[4], nn[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) tpixel(k0 + u * BLOCK + lane, key[u], pp[u]);
            if (knn2 || hsh) {
                auto search = [&](uint32_t key, int pix) {
                    int X, Y, wuv;
                    const int j = pix / s.W;
                    mark_params(s, pix - j * s.W, j, (int)(key >> 16), &X, &Y, &wuv);
                    return knn2 ? scan_nn(s, X, Y, 16 * (int)(key >> 16)) : hash_nn(s, X, Y, 16 * (int)(key >> 16));
                };
#pragma unroll
                for (int u = 0; u < 4; ++u) nn[u] = key[u] != kEmptyKey ? search(key[u], pp[u]) : -1;
            } else {
                // every lane loads (a clamped pixel, entry 0 of the table when
                // the depth has no entry) and keeps what its key selects
                int2 th[4];
                bool ok[4];
                int e[4], t[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) th[u] = gld(s.thdr + (uint32_t)pp[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    e[u] = (int)(key[u] >> 16) - (th[u].y & 0xFFFF);
                    ok[u] = key[u] != kEmptyKey && e[u] >= 0 && e[u] < (int)((uint32_t)th[u].y >> 16);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) t[u] = gld(s.tnn + (uint32_t)(ok[u] ? th[u].x + e[u] : 0));
#pragma unroll
                for (int u = 0; u < 4; ++u) nn[u] = ok[u] ? t[u] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (k0 + u * BLOCK < tpx) rstep(key[u] != kEmptyKey, k0 + u * BLOCK + lane, pp[u], nn[u]);
        }
        if (qc > 0) flush_r(qc);
        __syncthreads();

        // 4. J_o: observed points in V(O); explained iff some rendered point
        //    keyed it.  In RGB mode the key names the nearest rendered point,
        //    and the explained points are colour-tested through the wave's
        //    queue.  V rows above the J_o region go with the first band, rows
        //    below it with the last.
        const int ra = first ? in.vy0 : by0;
        const int rb = b == nb - 1 ? in.vy0 + in.vh : by0 + bh;
        const int rpx = max(rb - ra, 0) * in.vw;
        const float vinv = 1.0f / (float)max(in.vw, 1);
        auto flush_o = [&](int n) {
            wave_lds_sync();
            bool cout = false;
            if (lane < n) {
                const int2 e = q[lane];
                const int pix = e.x, kr = e.y;
                float4 lr;
                if (labs) {
                    lr = gld(labs + kr);       // every keying point is an inlier of the first band
                } else {
                    const uint32_t key = tld<G>(tile + kr);
                    const int ty = tile_row<G>(kr, in.tw, tinv), tx = kr - __mul24(ty, in.tw);
                    lr = srgb_to_lab(triangle_colour(s, m, P, (int)(key & 0xFFFFu), in.tx0 + tx, in.ty0 + ty));
                }
                cout = ciede2000(gld(s.olab + pix), lr) > s.tau;
                if (of) of[pix] = cout ? 3 : 1;
            }
            cO += wave_popc(cout);
        };
        // V pixel of the region's index k (clamped into the region) and its point
        auto vpixel = [&](int k, int &i, int &j) {
            const int kc = min(k, rpx - 1);
            const int vy = window_row(kc, in.vw, vinv), vx = kc - vy * in.vw;
            i = in.vx0 + vx;
            j = ra + vy;
            return j * s.W + i;
        };
        auto vtest = [&](bool live, int i, int j, int pix, int3 qo) {
            bool inq = false, out = false, need = false;
            int kr = 0;
            if (live) {
                if (qo.z != kNoPoint) {
                    const int dp = qo.z >> 4;
                    inq = label_mode ? (gld(s.labels + pix) == it.label) : in_volume(m, P, qo.x, qo.y, dp, dl, cyl);
                    typename K::T nk = K::kEmpty;
                    bool expl = false;
                    const int jx = i - in.jx0, jy = j - by0;
                    if (inq && jx >= 0 && jx < in.jw && jy >= 0 && jy < bh) {
                        if (nnm) {
                            expl = Marks<KG>::test(bits, jy * in.jw + jx);
                        } else {
                            nk = K::load(keys + jy * in.jw + jx);
                            expl = nk != K::kEmpty;
                        }
                    }
                    out = inq && !expl;
                    if (of && inq && (!expl || !ocol)) of[pix] = expl ? 1 : 2;
                    need = ocol && inq && expl;
                    kr = K::index(nk);
                }
            }
            cQ += wave_popc(inq);
            cO += wave_popc(out);
            if (ocol) {
                const unsigned long long mq = __ballot(need);
                if (need) q[qc + lane_rank(mq)] = make_int2(pix, kr);
                qc += __popcll(mq);
                if (qc >= 64) {
                    flush_o(64);
                    wave_lds_sync();
                    if (64 + lane < qc) q[lane] = q[64 + lane];
                    qc -= 64;
                }
            }
        };
        qc = 0;
        // four chunks a turn, every point loaded before any is tested
        for (int k0 = wave * 64; k0 < rpx; k0 += 4 * BLOCK) {
            int ii[4], jj[4], pp[4];
            int3 qq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pp[u] = vpixel(k0 + u * BLOCK + lane, ii[u], jj[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) qq[u] = opt_at(ms.opt, (uint32_t)pp[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (k0 + u * BLOCK < rpx) vtest(k0 + u * BLOCK + lane < rpx, ii[u], jj[u], pp[u], qq[u]);
        }
        if (qc > 0) flush_o(qc);
    }

    if (lane == 0) {
        atomicAdd(&cnt[0], cR);
        atomicAdd(&cnt[1], cO);
        atomicAdd(&cnt[2], cL);
        atomicAdd(&cnt[3], cQ);
    }
    __syncthreads();
    if (tid == 0) {
        it.jr[in.local] = cnt[0];
        it.jo[in.local] = cnt[1];
        if (it.nr) it.nr[in.local] = cnt[2];
        if (it.nq) it.nq[in.local] = cnt[3];
    }
    __syncthreads();
}

// Persistent scoring kernel for one size class.  G: the tile lives in
// device memory instead of LDS; KG: the J_o keys live in device memory
// (64-bit) instead of LDS (32-bit, after the tile).  RGB: the colour term is
// compiled in; PV: the paper's own variants, J_o by nearest-neighbour marking
// and the kNN II scan, are compiled in (each taken per scene).  Work-groups
// take the class's poses in turn.
template <int BLOCK, bool G, bool KG, bool RGB, bool PV>
__global__ __launch_bounds__(BLOCK, 4) void score_kernel(Work w, int cls)
{
    extern __shared__ uint32_t smem[];
    __shared__ int cnt[4];
    __shared__ int2 wq[BLOCK / 64 * 128];   // per-wave work queues of phases 3 and 4
    __shared__ int next;
    uint32_t *slot = w.gscratch + w.slot_base[cls] + (size_t)blockIdx.x * w.slot_words[cls];
    float4 *labs = RGB && w.lab ? w.lab + w.lab_base[cls] + (size_t)blockIdx.x * w.lab_px[cls] : nullptr;
    // Ordered lists are cut into image strips, one per XCD: a work-group
    // first takes the poses of its own XCD's strip (work-groups are
    // dispatched to the XCDs in turn), so each XCD's L2 holds one part of
    // the scene, then helps with the other strips.  Within a segment poses
    // come through a shared cursor, costliest first.
    const int home = blockIdx.x % kNumStrips;
    for (int h = 0; h < kNumStrips; ++h) {
        const int strip = (home + h) % kNumStrips;
        const int seg = cls * kNumStrips + strip;
        int start = 0, len;
        if (w.sort) {
            start = w.counts[kCntSegStart + seg];
            len = w.counts[kCntSegLen + seg];
        } else {
            len = strip == 0 ? w.counts[kCntClass + cls] : 0;
        }
        if (len == 0) continue;
        // The loop is headed by a wave-uniform value (readfirstlane of the
        // LDS copy) and no branch on the thread index: with a divergent
        // `if (tid == 0)` fetch at its top the compiler may send thread 0
        // alone round an outer loop to fetch while the other lanes pass the
        // barrier without it.  score_pose ends with a barrier, so every wave
        // has read `next` before thread 0 writes it again.
        if (threadIdx.x == 0) next = atomicAdd(&w.counts[kCntNext + seg], 1);
        __syncthreads();
        for (int i = __builtin_amdgcn_readfirstlane(next); i < len;) {
            const int p = __builtin_amdgcn_readfirstlane(w.lists[cls * w.cap_poses + start + i]);
            uint32_t *tile = G ? slot : smem;
            typename KeyOf<KG>::T *keys;
            if constexpr (KG)
                keys = reinterpret_cast<unsigned long long *>(G ? slot + w.dev_tile_words : slot);
            else
                keys = smem + w.info[p].tw * w.info[p].th;
            score_pose<BLOCK, G, KG, RGB, PV>(w, p, tile, keys, labs, cnt, wq);
            if (threadIdx.x == 0) next = atomicAdd(&w.counts[kCntNext + seg], 1);
            __syncthreads();
            i = __builtin_amdgcn_readfirstlane(next);
        }
        // every wave has read the segment's last `next` before the next
        // segment's fetch overwrites it
        __syncthreads();
    }
}

// ------------------------------------------------------------------ setup

__global__ void zero_counts_kernel(int *counts)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kCounterInts) counts[k] = 0;
}

// Cost bucket of a pose from its raster tile, J_o region and triangle
// count, weighted as the per-pose work of rasterizing and searching.
__device__ __forceinline__ int cost_bucket(int tile_px, int j_px, int nt)
{
    const long long est = 3LL * tile_px + j_px + nt / 5 + 1;
    const int lg = 63 - __clzll(est);
    return min(max(lg - 4, 0), kNumBuckets - 1);
}

// Regions and footprint class of global pose p; returns its order key
// (class * kNumStrips + strip) * kNumBuckets + sub-key.
__device__ int classify_pose(const Work &w, int p)
{
    // the item holding global pose p: the last one with first <= p
    int lo = 0, hi = w.hdr->n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (w.items[mid].first <= p) lo = mid;
        else hi = mid - 1;
    }
    const ItemDev &it = w.items[lo];
    const SceneDev &s = w.scenes[it.scene];
    const MeshDev &m = w.meshes[it.mesh];
    float P[12];
    for (int k = 0; k < 12; ++k) P[k] = it.poses[12 * (size_t)(p - it.first) + k];
    PoseInfo in;
    in.item = lo;
    in.local = p - it.first;
    double umin, umax, vmin, vmax, zmin, zmax;
    // Raster tile: every drawn vertex has Zc >= 100 and lies in the AABB.
    project_box(P, m.lo, m.hi, 0.0, s, &umin, &umax, &vmin, &vmax, &zmin, &zmax);
    if (zmin >= 100.0) {
        clip_box(umin, umax, vmin, vmax, s.W, s.H, &in.tx0, &in.ty0, &in.tw, &in.th);
    } else if (zmax < 99.999) {
        in.tx0 = in.ty0 = in.tw = in.th = 0;
    } else {
        in.tx0 = in.ty0 = 0;
        in.tw = s.W;
        in.th = s.H;
    }
    // J_o region: observed pixels whose point may lie in the inflated AABB.
    if ((s.flags & (3u << 4)) == (2u << 4)) {
        in.vx0 = it.vbox[0];
        in.vy0 = it.vbox[1];
        in.vw = it.vbox[2];
        in.vh = it.vbox[3];
    } else {
        project_box(P, m.lo, m.hi, (double)s.delta + 0.5, s, &umin, &umax, &vmin, &vmax, &zmin, &zmax);
        if (zmin > 0.5) {
            clip_box(umin, umax, vmin, vmax, s.W, s.H, &in.vx0, &in.vy0, &in.vw, &in.vh);
        } else if (zmax <= 0.0) {
            in.vx0 = in.vy0 = in.vw = in.vh = 0;
        } else {
            in.vx0 = in.vy0 = 0;
            in.vw = s.W;
            in.vh = s.H;
        }
    }
    // J_o region: the part of the V region that a rendered point's
    // neighbours can reach (the tile dilated by the neighbour window).
    in.jx0 = max(in.vx0, in.tx0 - s.wtx);
    in.jy0 = max(in.vy0, in.ty0 - s.wty);
    const int jx1 = min(in.vx0 + in.vw - 1, in.tx0 + in.tw - 1 + s.wtx);
    const int jy1 = min(in.vy0 + in.vh - 1, in.ty0 + in.th - 1 + s.wty);
    in.jw = (in.tw > 0 && jx1 >= in.jx0) ? jx1 - in.jx0 + 1 : 0;
    in.jh = (in.th > 0 && jy1 >= in.jy0) ? jy1 - in.jy0 + 1 : 0;
    if (in.jw == 0 || in.jh == 0) in.jw = in.jh = 0;
    w.info[p] = in;
    // LDS words: tile + 32-bit keys; 32-bit keys need d2 < 2^16 and tile
    // indices < 2^16, otherwise the pose is scored from device memory
    // (J_o by nearest-neighbour marking: a bitmap, one bit per pixel, with
    // no index to hold and no bands)
    const bool nnm = (s.flags & 64u) != 0;
    const int tile_words = in.tw * in.th;
    const int words = tile_words + (nnm ? (in.jw * in.jh + 31) / 32 : in.jw * in.jh);
    int cls = tile_words <= w.cap_large ? 2 : 3;
    if (it.key32 || nnm) {
        if (words <= w.cap_large) cls = words <= w.cap_small ? 0 : 1;
        else if (!nnm && w.key_bands && tile_words + in.jw <= w.cap_large) cls = 1;   // J_o keys in bands of rows
    }
    const int strip = min(max(((in.tx0 + in.tw / 2) * kNumStrips) / s.W, 0), kNumStrips - 1);
    // within a strip: costliest first for one scene; by scene group when the
    // launch spans several scenes, so an XCD works through a few scenes' data
    // at a time
    const int ns = w.hdr->n_scenes;
    const int sub = ns > 1 ? (it.scene * kNumBuckets) / ns : kNumBuckets - 1 - cost_bucket(tile_words, in.jw * in.jh, m.nt);
    const int order = (cls * kNumStrips + strip) * kNumBuckets + sub;
    w.info[p].order = order;
    return order;
}

// Classify every pose.  Counts are gathered per work-group in LDS and added
// to the launch counters once per work-group and key.  Without ordering,
// each class list is filled in set-up order (one segment per class).
__global__ __launch_bounds__(256) void setup_kernel(Work w)
{
    __shared__ int lcnt[kNumOrders];
    __shared__ int lcls[kNumClasses], lbase[kNumClasses];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    for (int k = threadIdx.x; k < kNumOrders; k += blockDim.x) lcnt[k] = 0;
    if (threadIdx.x < kNumClasses) lcls[threadIdx.x] = 0;
    __syncthreads();
    int order = -1, local = 0;
    if (p < w.hdr->n_poses) {
        order = classify_pose(w, p);
        if (w.sort) atomicAdd(&lcnt[order], 1);
        else local = atomicAdd(&lcls[order / (kNumStrips * kNumBuckets)], 1);
    }
    __syncthreads();
    if (w.sort) {
        for (int k = threadIdx.x; k < kNumOrders; k += blockDim.x) {
            const int c = lcnt[k];
            if (c) {
                atomicAdd(&w.counts[kCntBucket + k], c);
                atomicAdd(&w.counts[kCntClass + k / (kNumStrips * kNumBuckets)], c);
            }
        }
        return;
    }
    if (threadIdx.x < kNumClasses) {
        const int c = lcls[threadIdx.x];
        lbase[threadIdx.x] = c ? atomicAdd(&w.counts[kCntClass + threadIdx.x], c) : 0;
    }
    __syncthreads();
    if (order >= 0) {
        const int cls = order / (kNumStrips * kNumBuckets);
        w.lists[cls * w.cap_poses + lbase[cls] + local] = p;
    }
}

// Place each pose in its class list: by image strip, then by the sub-key
// (cost bucket, costliest first, or scene group), ascending (order within a
// key is arbitrary: every pose is scored independently).  The first work-group also records each (class, strip)
// segment.  Slots are taken per work-group and key, then handed out in LDS.
__global__ __launch_bounds__(256) void order_kernel(Work w)
{
    __shared__ int seg[kNumSegs];
    __shared__ int base[kNumOrders], lcnt[kNumOrders], lbase[kNumOrders];
    const int t = threadIdx.x;
    if (t < kNumSegs) {
        int n = 0;
        for (int b = 0; b < kNumBuckets; ++b) n += w.counts[kCntBucket + t * kNumBuckets + b];
        seg[t] = n;
    }
    for (int k = t; k < kNumOrders; k += blockDim.x) lcnt[k] = 0;
    __syncthreads();
    for (int k = t; k < kNumOrders; k += blockDim.x) {
        const int sg = k / kNumBuckets, b = k % kNumBuckets;
        const int cls = sg / kNumStrips, strip = sg % kNumStrips;
        int off = 0;
        for (int s2 = 0; s2 < strip; ++s2) off += seg[cls * kNumStrips + s2];
        for (int b2 = 0; b2 < b; ++b2) off += w.counts[kCntBucket + sg * kNumBuckets + b2];
        base[k] = off;
    }
    if (blockIdx.x == 0 && t < kNumSegs) {
        const int cls = t / kNumStrips, strip = t % kNumStrips;
        int off = 0;
        for (int s2 = 0; s2 < strip; ++s2) off += seg[cls * kNumStrips + s2];
        w.counts[kCntSegStart + t] = off;
        w.counts[kCntSegLen + t] = seg[t];
    }
    const int p = blockIdx.x * blockDim.x + t;
    const bool valid = p < w.hdr->n_poses;
    int order = 0, local = 0;
    if (valid) {
        order = w.info[p].order;
        local = atomicAdd(&lcnt[order], 1);
    }
    __syncthreads();
    for (int k = t; k < kNumOrders; k += blockDim.x) {
        const int c = lcnt[k];
        lbase[k] = c ? atomicAdd(&w.counts[kCntFill + k], c) : 0;
    }
    __syncthreads();
    if (valid) {
        const int cls = order / (kNumStrips * kNumBuckets);
        w.lists[cls * w.cap_poses + base[order] + lbase[order] + local] = p;
    }
}

// ------------------------------------------------------------------ scene prep

__global__ void scene_points_kernel(SceneDev s, const uint8_t *rgb, int4 *opt, float4 *olab)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.W * s.H) return;
    const int j = k / s.W, i = k - j * s.W;
    const int d = s.depth[k];
    int4 q = make_int4(0, 0, kNoPoint, 0);
    if (d > 0) {
        q.x = (int)rint(s.kx[i] * (double)d);
        q.y = (int)rint(s.ky[j] * (double)d);
        q.z = 16 * d;
    }
    opt[k] = q;
    if (olab) {
        const uint32_t c = (uint32_t)rgb[3 * (size_t)k] | ((uint32_t)rgb[3 * (size_t)k + 1] << 8)
                           | ((uint32_t)rgb[3 * (size_t)k + 2] << 16);
        olab[k] = srgb_to_lab(c);
    }
}

// ------------------------------------------------------------------ NN table

// Row pass of the window min/max of valid observed depths: min | max << 16.
__global__ void table_rows_kernel(SceneDev s, uint32_t *tmp)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.W * s.H) return;
    const int j = k / s.W, i = k - j * s.W;
    int mn = 0xFFFF, mx = 0;
    for (int ii = max(i - s.wtx, 0); ii <= min(i + s.wtx, s.W - 1); ++ii) {
        const int d = s.depth[j * s.W + ii];
        if (d == 0) continue;
        mn = min(mn, d);
        mx = max(mx, d);
    }
    tmp[k] = (uint32_t)mn | ((uint32_t)mx << 16);
}

// Column pass: the depths a rendered point at this pixel may have and still
// find an observed point within delta: [min - dzmm, max + dzmm].
__global__ void table_cols_kernel(SceneDev s, const uint32_t *tmp, int2 *thdr)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.W * s.H) return;
    const int j = k / s.W, i = k - j * s.W;
    int mn = 0xFFFF, mx = 0;
    for (int jj = max(j - s.wty, 0); jj <= min(j + s.wty, s.H - 1); ++jj) {
        const uint32_t v = tmp[jj * s.W + i];
        mn = min(mn, (int)(v & 0xFFFFu));
        mx = max(mx, (int)(v >> 16));
    }
    int lo = 0, n = 0;
    if (mx > 0) {
        lo = max(1, mn - s.dzmm);
        const int hi = min(65534, mx + s.dzmm);
        n = hi - lo + 1;
    }
    thdr[k] = make_int2(0, lo | (n << 16));
}

// Exclusive scan of the per-pixel entry counts (thdr[].y >> 16) into
// thdr[].x, in three passes over blocks of kScanBlock pixels: block sums,
// a one-work-group scan of the block sums (with the grand total), and the
// scan inside each block offset by its block's start.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ long long block_exclusive_scan256(long long v, long long *total)
{
    __shared__ long long wsum[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    long long x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const long long y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    long long before = 0, all = 0;
    for (int k = 0; k < 4; ++k) {
        if (k < wv) before += wsum[k];
        all += wsum[k];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ __launch_bounds__(256) void table_block_sums_kernel(int N, const int2 *thdr, long long *blk)
{
    const int base = blockIdx.x * kScanBlock + 4 * threadIdx.x;
    long long v = 0;
    for (int u = 0; u < 4; ++u)
        if (base + u < N) v += (long long)((uint32_t)thdr[base + u].y >> 16);
    long long total;
    (void)block_exclusive_scan256(v, &total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void table_block_scan_kernel(int nblk, long long *blk, long long *total)
{
    // 256 threads, each a contiguous run of the block sums
    const int chunk = (nblk + 255) / 256;
    const int a = threadIdx.x * chunk, b = min(a + chunk, nblk);
    long long v = 0;
    for (int k = a; k < b; ++k) v += blk[k];
    long long all;
    long long run = block_exclusive_scan256(v, &all);
    for (int k = a; k < b; ++k) {
        const long long x = blk[k];
        blk[k] = run;
        run += x;
    }
    if (threadIdx.x == 0) *total = all;
}

__global__ __launch_bounds__(256) void table_block_apply_kernel(int N, int2 *thdr, const long long *blk)
{
    const int base = blockIdx.x * kScanBlock + 4 * threadIdx.x;
    int n[4];
    long long v = 0;
    for (int u = 0; u < 4; ++u) {
        n[u] = base + u < N ? (int)((uint32_t)thdr[base + u].y >> 16) : 0;
        v += n[u];
    }
    long long total;
    long long run = blk[blockIdx.x] + block_exclusive_scan256(v, &total);
    for (int u = 0; u < 4; ++u)
        if (base + u < N) {
            thdr[base + u].x = (int)run;     // the total is checked to fit 31 bits before any use
            run += n[u];
        }
}

// ------------------------------------------------------------------ voxel hash

__global__ void fill_zero_kernel(int *a, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) a[k] = 0;
}

__device__ __forceinline__ int point_bucket(const SceneDev &s, int4 q)
{
    return cell_bucket(q.x >> s.hshift, q.y >> s.hshift, q.z >> s.hshift, s.hbits);
}

// Points per bucket.
__global__ void hash_count_kernel(SceneDev s, int *count)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.W * s.H) return;
    const int4 q = s.opt[k];
    if (q.z == kNoPoint) return;
    atomicAdd(count + point_bucket(s, q), 1);
}

// Block sums of the bucket counts, blocks of kScanBlock.
__global__ __launch_bounds__(256) void hash_block_sums_kernel(int M, const int *count, long long *blk)
{
    const int base = blockIdx.x * kScanBlock + 4 * threadIdx.x;
    long long v = 0;
    for (int u = 0; u < 4; ++u)
        if (base + u < M) v += count[base + u];
    long long total;
    (void)block_exclusive_scan256(v, &total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

// Bucket starts: the exclusive scan of the counts, and start[M] = all points.
__global__ __launch_bounds__(256) void hash_block_apply_kernel(int M, const int *count, const long long *blk,
                                                               int *start)
{
    const int base = blockIdx.x * kScanBlock + 4 * threadIdx.x;
    int n[4];
    long long v = 0;
    for (int u = 0; u < 4; ++u) {
        n[u] = base + u < M ? count[base + u] : 0;
        v += n[u];
    }
    long long total;
    long long run = blk[blockIdx.x] + block_exclusive_scan256(v, &total);
    for (int u = 0; u < 4; ++u) {
        if (base + u < M) start[base + u] = (int)run;
        run += n[u];
        if (base + u == M - 1) start[M] = (int)run;
    }
}

// Each point into its bucket's range (the order inside a bucket is free:
// queries keep the smallest (d^2, pixel)); count is consumed.
__global__ void hash_scatter_kernel(SceneDev s, int *count, int4 *pts)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.W * s.H) return;
    const int4 q = s.opt[k];
    if (q.z == kNoPoint) return;
    const int b = point_bucket(s, q);
    const int slot = atomicSub(count + b, 1) - 1;
    pts[s.hstart[b] + slot] = make_int4(q.x, q.y, q.z, k);
}

hipError_t launch_hash_build(const SceneDev &s, int *count, long long *blk, hipStream_t st)
{
    const int N = s.W * s.H, M = 1 << s.hbits;
    const int nblk = table_scan_blocks(M);
    fill_zero_kernel<<<(M + 255) / 256, 256, 0, st>>>(count, M);
    hash_count_kernel<<<(N + 255) / 256, 256, 0, st>>>(s, count);
    hash_block_sums_kernel<<<nblk, 256, 0, st>>>(M, count, blk);
    table_block_scan_kernel<<<1, 256, 0, st>>>(nblk, blk, blk + nblk);
    hash_block_apply_kernel<<<nblk, 256, 0, st>>>(M, count, blk, const_cast<int *>(s.hstart));
    hash_scatter_kernel<<<(N + 255) / 256, 256, 0, st>>>(s, count, const_cast<int4 *>(s.hpts));
    return hipGetLastError();
}

// Entries of one pixel's range handled per pass of the fill kernel.
constexpr int kFillChunk = 256;


// One wave per pixel.  An observed point q can lie within delta of a
// rendered point at this pixel only at depths within dzmm of q's own, so the
// lanes take the observed points of the pixel's window and each visits just
// the depths of the range that q can reach, min-combining (squared
// distance, pixel index) into that depth's entry in LDS.  The entries'
// back-projected (X, Y) are computed once per pass.  Ranges longer than
// kFillChunk are filled in several passes.
__global__ __launch_bounds__(256) void table_fill_kernel(SceneDev s, int32_t *tnn, long long cap)
{
    __shared__ unsigned long long acc[4][kFillChunk];
    __shared__ int2 exy[4][kFillChunk];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int a = blockIdx.x * 4 + wv;
    if (a >= s.W * s.H) return;                 // no block-wide barrier below
    const int2 th = s.thdr[a];
    const int lo = th.y & 0xFFFF, n = (int)((uint32_t)th.y >> 16);
    if (n == 0) return;
    const int j = a / s.W, i = a - j * s.W;
    const double kxi = s.kx[i], kyj = s.ky[j];
    const float dl = s.delta + 0.25f;
    for (int c0 = 0; c0 < n; c0 += kFillChunk) {
        const int cn = min(kFillChunk, n - c0);
        const int dmin = lo + c0, dmax = lo + c0 + cn - 1;
        for (int e = lane; e < cn; e += 64) {
            acc[wv][e] = ~0ULL;
            exy[wv][e] = make_int2((int)rint(kxi * (double)(dmin + e)), (int)rint(kyj * (double)(dmin + e)));
        }
        wave_lds_sync();
        // the window of the pass's smallest depth is the widest one
        const float iz = window_inv(dmin, dl);
        const int wu = window_half(gld(s.ax + i), iz, s.W);
        const int wvv = window_half(gld(s.ay + j), iz, s.H);
        const int i0 = max(i - wu, 0), i1 = min(i + wu, s.W - 1);
        const int j0 = max(j - wvv, 0), j1 = min(j + wvv, s.H - 1);
        const int ww = i1 - i0 + 1;
        const int ws = ww * (j1 - j0 + 1);
        const float inv = 1.0f / (float)ww;
        const int dlo = dmin - s.dzmm, dhi = dmax + s.dzmm;
        for (int q = lane; q < ws; q += 64) {
            const int qy = window_row(q, ww, inv);
            const int pix = (j0 + qy) * s.W + i0 + (q - qy * ww);
            const int4 xy = gld(s.opt + pix);
            const int dp = xy.z >> 4;
            if (xy.z == kNoPoint || dp < dlo || dp > dhi) continue;
            const int ea = max(dp - s.dzmm, dmin) - dmin, eb = min(dp + s.dzmm, dmax) - dmin;
            for (int e = ea; e <= eb; ++e) {
                const int dz = 16 * dp - 16 * (dmin + e);
                const int2 r = exy[wv][e];
                const int dx = xy.x - r.x, dy = xy.y - r.y;
                if (max(max(abs(dz), abs(dx)), abs(dy)) > s.dq) continue;
                const int d2 = __mul24(dx, dx) + __mul24(dy, dy) + __mul24(dz, dz);
                if (d2 > s.dq2) continue;
                atomicMin(&acc[wv][e], ((unsigned long long)d2 << 32) | (uint32_t)pix);
            }
        }
        wave_lds_sync();
        for (int e = lane; e < cn; e += 64) {
            const unsigned long long best = acc[wv][e];
            if ((long long)th.x + c0 + e < cap) tnn[th.x + c0 + e] = best == ~0ULL ? -1 : (int32_t)(best & 0xFFFFFFFFu);
        }
        wave_lds_sync();
    }
}

int table_scan_blocks(int n_pixels) { return (n_pixels + kScanBlock - 1) / kScanBlock; }

hipError_t launch_table_ranges(const SceneDev &s, uint32_t *tmp, int2 *thdr, long long *total, long long *blk,
                               hipStream_t st)
{
    const int N = s.W * s.H;
    const int nblk = table_scan_blocks(N);
    table_rows_kernel<<<(N + 255) / 256, 256, 0, st>>>(s, tmp);
    table_cols_kernel<<<(N + 255) / 256, 256, 0, st>>>(s, tmp, thdr);
    table_block_sums_kernel<<<nblk, 256, 0, st>>>(N, thdr, blk);
    table_block_scan_kernel<<<1, 256, 0, st>>>(nblk, blk, total);
    table_block_apply_kernel<<<nblk, 256, 0, st>>>(N, thdr, blk);
    return hipGetLastError();
}

hipError_t launch_table_fill(const SceneDev &s, int32_t *tnn, long long cap, hipStream_t st)
{
    const int N = s.W * s.H;
    table_fill_kernel<<<(N + 3) / 4, 256, 0, st>>>(s, tnn, cap);
    return hipGetLastError();
}

// ------------------------------------------------------------------ render (inspection)

__global__ __launch_bounds__(256) void render_kernel(SceneDev s, MeshDev m, const float *poses, uint32_t *keys,
                                                     uint16_t *depth, uint8_t *rgb, int32_t *tri)
{
    const int p = blockIdx.x;
    const size_t N = (size_t)s.W * s.H;
    uint32_t *K = keys + p * N;
    float P[12];
    for (int k = 0; k < 12; ++k) P[k] = poses[12 * (size_t)p + k];
    for (size_t k = threadIdx.x; k < N; k += 256) tst<true>(K + k, kEmptyKey);
    __syncthreads();
    for (int t0 = 0; t0 < m.nt; t0 += 256) {
        const int t = t0 + threadIdx.x;
        if (t < m.nt) raster_triangle<true>(s, m, P, t, 0, 0, s.W, s.H, K);
    }
    __syncthreads();
    for (size_t k = threadIdx.x; k < N; k += 256) {
        const uint32_t key = tld<true>(K + k);
        const bool e = key == kEmptyKey;
        depth[p * N + k] = e ? 0 : (uint16_t)(key >> 16);
        if (tri) tri[p * N + k] = e ? -1 : (int32_t)(key & 0xFFFFu);
        if (rgb) {
            uint32_t c = 0;
            if (!e && m.vrgb) {
                const int j = (int)(k / s.W), i = (int)(k - (size_t)j * s.W);
                c = triangle_colour(s, m, P, (int)(key & 0xFFFFu), i, j);
            }
            rgb[3 * (p * N + k)] = (uint8_t)(c & 255u);
            rgb[3 * (p * N + k) + 1] = (uint8_t)((c >> 8) & 255u);
            rgb[3 * (p * N + k) + 2] = (uint8_t)((c >> 16) & 255u);
        }
    }
}

// ------------------------------------------------------------------ argmin

// Per work item: the minimum of J = J_r + J_o over its poses, the lowest
// pose index among ties; best[2 item] = index, best[2 item + 1] = J.
__global__ __launch_bounds__(1024) void item_argmin_kernel(Work w)
{
    __shared__ unsigned long long red[16];
    const int item = blockIdx.x;
    if (item >= w.hdr->n_items) return;
    const ItemDev &it = w.items[item];
    unsigned long long best = ~0ULL;
    for (int k = threadIdx.x; k < it.n; k += 1024) {
        const unsigned long long key = ((unsigned long long)(uint32_t)(it.jr[k] + it.jo[k]) << 32) | (uint32_t)k;
        best = key < best ? key : best;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x < 64) {
        best = threadIdx.x < 16 ? red[threadIdx.x] : ~0ULL;
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(best, off);
            best = o < best ? o : best;
        }
        if (threadIdx.x == 0) {
            w.best[2 * item] = best == ~0ULL ? -1 : (int32_t)(best & 0xFFFFFFFFu);
            w.best[2 * item + 1] = best == ~0ULL ? -1 : (int32_t)(best >> 32);
        }
    }
}

// ------------------------------------------------------------------ launchers

hipError_t upload_colour_table(const float *lin256)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lin), lin256, 256 * sizeof(float));
}

hipError_t launch_scene_prep(const SceneDev &s, const uint8_t *rgb_dev, int4 *opt, float4 *olab, hipStream_t st)
{
    const int N = s.W * s.H;
    scene_points_kernel<<<(N + 255) / 256, 256, 0, st>>>(s, rgb_dev, opt, olab);
    return hipGetLastError();
}

template <int BLOCK, bool G, bool KG, bool RGB, bool PV>
static hipError_t launch_one(const Work &w, int cls, int grid, int lds_words, hipStream_t st)
{
    score_kernel<BLOCK, G, KG, RGB, PV><<<grid, BLOCK, (size_t)lds_words * 4, st>>>(w, cls);
    return hipGetLastError();
}

template <bool RGB, bool PV>
static hipError_t prepare_t(int lds_per_group, int static_bytes[3])
{
    struct K {
        const void *f;
        int slot;
    };
    const K ks[] = {{(const void *)score_kernel<256, false, false, RGB, PV>, 0},
                    {(const void *)score_kernel<512, false, false, RGB, PV>, 1},
                    {(const void *)score_kernel<1024, false, false, RGB, PV>, 2},
                    {(const void *)score_kernel<1024, false, true, RGB, PV>, 2}};
    for (const K &k : ks) {
        hipFuncAttributes a{};
        hipError_t e = hipFuncGetAttributes(&a, k.f);
        if (e != hipSuccess) return e;
        const int st = (int)a.sharedSizeBytes;
        static_bytes[k.slot] = max(static_bytes[k.slot], st);
        e = hipFuncSetAttribute(k.f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_per_group - st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t prepare_score_kernels(int lds_per_group, int static_bytes[3])
{
    static_bytes[0] = static_bytes[1] = static_bytes[2] = 0;
    hipError_t e = prepare_t<false, false>(lds_per_group, static_bytes);
    if (e == hipSuccess) e = prepare_t<true, false>(lds_per_group, static_bytes);
    if (e == hipSuccess) e = prepare_t<false, true>(lds_per_group, static_bytes);
    return e == hipSuccess ? prepare_t<true, true>(lds_per_group, static_bytes) : e;
}

template <bool RGB, bool PV>
static hipError_t launch_class_t(const Work &w, const LaunchCfg &c, int cls, hipStream_t st)
{
    switch (cls) {
    case 0:
        return c.small_block == 256 ? launch_one<256, false, false, RGB, PV>(w, 0, c.grid[0], c.cap_small, st)
                                    : launch_one<512, false, false, RGB, PV>(w, 0, c.grid[0], c.cap_small, st);
    case 1: return launch_one<1024, false, false, RGB, PV>(w, 1, c.grid[1], c.cap_large, st);
    case 2: return launch_one<1024, false, true, RGB, PV>(w, 2, c.grid[2], c.cap_large, st);
    default: return launch_one<256, true, true, RGB, PV>(w, 3, c.grid[3], 0, st);
    }
}

hipError_t launch_setup(const Work &w, int poses_grid, hipStream_t st)
{
    zero_counts_kernel<<<(kCounterInts + 255) / 256, 256, 0, st>>>(w.counts);
    setup_kernel<<<(poses_grid + 255) / 256, 256, 0, st>>>(w);
    if (w.sort) order_kernel<<<(poses_grid + 255) / 256, 256, 0, st>>>(w);
    return hipGetLastError();
}

hipError_t launch_score_class(const Work &w, const LaunchCfg &c, int cls, bool any_rgb, bool any_pv, hipStream_t st)
{
    if (any_pv)
        return any_rgb ? launch_class_t<true, true>(w, c, cls, st) : launch_class_t<false, true>(w, c, cls, st);
    return any_rgb ? launch_class_t<true, false>(w, c, cls, st) : launch_class_t<false, false>(w, c, cls, st);
}

hipError_t launch_item_argmin(const Work &w, int items_grid, hipStream_t st)
{
    item_argmin_kernel<<<items_grid, 1024, 0, st>>>(w);
    return hipGetLastError();
}

struct DescArg {
    uint4 w[kDescArgBytes / 16];
};

__global__ void desc_write_kernel(DescArg a, int n16, uint4 *dst)
{
    if ((int)threadIdx.x < n16) dst[threadIdx.x] = a.w[threadIdx.x];
}

hipError_t launch_desc_write(const void *bytes, size_t n, void *dst, hipStream_t st)
{
    if (n > (size_t)kDescArgBytes) return hipErrorInvalidValue;
    DescArg a{};
    memcpy(&a, bytes, n);
    desc_write_kernel<<<1, kDescArgBytes / 16, 0, st>>>(a, (int)((n + 15) / 16), (uint4 *)dst);
    return hipGetLastError();
}

hipError_t launch_render(const SceneDev &s, const MeshDev &m, const float *poses, int n, uint32_t *keys,
                         uint16_t *depth, uint8_t *rgb, int32_t *tri, hipStream_t st)
{
    render_kernel<<<n, 256, 0, st>>>(s, m, poses, keys, depth, rgb, tri);
    return hipGetLastError();
}

}  // namespace perch
