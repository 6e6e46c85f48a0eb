// gfx950 kernels for PERCH 2.0 pose scoring.
//
// Per candidate pose (Sec. IV-A "Parallel Rendering" / "Parallel Cost
// Computation", Eq. 1-4):
//   1. rasterize the mesh into an LDS-resident tile of 32-bit keys
//      (depth mm << 16 | triangle index), min-combined with ds_min_u32;
//   2. resolve: drop occluders (Eq. 3, C from the observed depth) and pixels
//      off the downsampling grid;
//   3. J_r: radius / nearest-neighbour search of each rendered point in the
//      observed cloud, restricted to the pixel window that can hold a point
//      within delta and pruned by per-8x8-block depth ranges;
//   4. J_o: for each observed pixel inside V(O), the same search against the
//      rendered tile;
//   5. RGB mode: CIEDE2000 of each point against its nearest neighbour
//      (Eq. 4), in binary32;
//   6. wave ballot + popcount of the outlier predicates.
// Geometry and depth use integer / binary64 arithmetic that is reproduced
// exactly by the CPU reference (no FMA contraction: built with
// -ffp-contract=off).

#include "perch_internal.h"

#include <math.h>

namespace perch {

__constant__ float c_lin[256];   // sRGB8 -> linear, rounded from binary64

// ------------------------------------------------------------------ geometry

struct Vtx {
    int U, V;      // 24.8 fixed point
    double iz;     // 1 / Zc
    int ok;
};

__device__ __forceinline__ Vtx project_vertex(const float *P, float4 v, const SceneDev &s)
{
    const double x = v.x, y = v.y, z = v.z;
    const double X = (((double)P[0] * x + (double)P[1] * y) + (double)P[2] * z) + (double)P[3];
    const double Y = (((double)P[4] * x + (double)P[5] * y) + (double)P[6] * z) + (double)P[7];
    const double Z = (((double)P[8] * x + (double)P[9] * y) + (double)P[10] * z) + (double)P[11];
    Vtx o;
    o.ok = 0;
    o.U = 0;
    o.V = 0;
    o.iz = 0.0;
    if (!(Z >= 100.0)) return o;
    o.iz = 1.0 / Z;
    const double u = (((double)s.fx * X) * o.iz) + (double)s.cx;
    const double w = (((double)s.fy * Y) * o.iz) + (double)s.cy;
    const double su = 256.0 * u, sv = 256.0 * w;
    if (!(fabs(su) <= 16777216.0) || !(fabs(sv) <= 16777216.0)) return o;
    o.U = (int)rint(su);
    o.V = (int)rint(sv);
    o.ok = 1;
    return o;
}

__device__ __forceinline__ long long edge_fn(int ax, int ay, int bx, int by, long long px, long long py)
{
    return (long long)(by - ay) * (px - ax) - (long long)(bx - ax) * (py - ay);
}

// covered iff E > 0, or E == 0 on a top-left edge  <=>  E >= bias
__device__ __forceinline__ long long edge_bias(int ax, int ay, int bx, int by)
{
    const int dy = by - ay, dx = bx - ax;
    return (dy > 0 || (dy == 0 && dx < 0)) ? 0 : 1;
}

// tile accessors: plain LDS traffic, or agent-scope atomics for global tiles
template <bool G>
__device__ __forceinline__ uint32_t tld(const uint32_t *p)
{
    if constexpr (G) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <bool G>
__device__ __forceinline__ void tst(uint32_t *p, uint32_t v)
{
    if constexpr (G) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
template <bool G>
__device__ __forceinline__ void tmin(uint32_t *p, uint32_t v)
{
    if constexpr (G) __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else atomicMin(p, v);
}
template <bool G>
__device__ __forceinline__ void tmax(uint32_t *p, uint32_t v)
{
    if constexpr (G) __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else atomicMax(p, v);
}

// Rasterize triangle t into the tile covering pixels [tx0, tx0+tw) x [ty0, ty0+th).
template <bool G>
__device__ __forceinline__ void raster_triangle(const SceneDev &s, const MeshDev &m, const float *P,
                                                int t, int tx0, int ty0, int tw, int th,
                                                uint32_t *tile)
{
    const int4 ix = m.tris[t];
    const Vtx a = project_vertex(P, m.verts[ix.x], s);
    const Vtx b = project_vertex(P, m.verts[ix.y], s);
    const Vtx c = project_vertex(P, m.verts[ix.z], s);
    if (!(a.ok & b.ok & c.ok)) return;
    const long long area = edge_fn(a.U, a.V, b.U, b.V, c.U, c.V);
    if (area <= 0) return;
    const int minU = min(a.U, min(b.U, c.U)), maxU = max(a.U, max(b.U, c.U));
    const int minV = min(a.V, min(b.V, c.V)), maxV = max(a.V, max(b.V, c.V));
    const int i0 = max(-((-minU) >> 8), tx0), i1 = min(maxU >> 8, tx0 + tw - 1);
    const int j0 = max(-((-minV) >> 8), ty0), j1 = min(maxV >> 8, ty0 + th - 1);
    if (i0 > i1 || j0 > j1) return;
    const long long px0 = 256LL * i0, py0 = 256LL * j0;
    long long r0 = edge_fn(b.U, b.V, c.U, c.V, px0, py0);
    long long r1 = edge_fn(c.U, c.V, a.U, a.V, px0, py0);
    long long r2 = edge_fn(a.U, a.V, b.U, b.V, px0, py0);
    const long long sx0 = 256LL * (c.V - b.V), sy0 = -256LL * (c.U - b.U);
    const long long sx1 = 256LL * (a.V - c.V), sy1 = -256LL * (a.U - c.U);
    const long long sx2 = 256LL * (b.V - a.V), sy2 = -256LL * (b.U - a.U);
    const long long b0 = edge_bias(b.U, b.V, c.U, c.V);
    const long long b1 = edge_bias(c.U, c.V, a.U, a.V);
    const long long b2 = edge_bias(a.U, a.V, b.U, b.V);
    const double farea = (double)area;
    for (int j = j0; j <= j1; ++j) {
        long long w0 = r0, w1 = r1, w2 = r2;
        uint32_t *row = tile + (size_t)(j - ty0) * tw;
        for (int i = i0; i <= i1; ++i) {
            if (w0 >= b0 && w1 >= b1 && w2 >= b2) {
                const double t0 = (double)w0 * a.iz, t1 = (double)w1 * b.iz, t2 = (double)w2 * c.iz;
                const double sum = (t0 + t1) + t2;
                const double d = rint(farea / sum);
                if (d >= 1.0 && d <= 65534.0)
                    tmin<G>(row + (i - tx0), ((uint32_t)d << 16) | (uint32_t)t);
            }
            w0 += sx0;
            w1 += sx1;
            w2 += sx2;
        }
        r0 += sy0;
        r1 += sy1;
        r2 += sy2;
    }
}

// Perspective-correct vertex colour of triangle t at pixel (i, j), rounded to sRGB8.
__device__ uint32_t triangle_colour(const SceneDev &s, const MeshDev &m, const float *P, int t, int i, int j)
{
    if (t < 0 || t >= m.nt) return 0;
    const int4 ix = m.tris[t];
    const Vtx a = project_vertex(P, m.verts[ix.x], s);
    const Vtx b = project_vertex(P, m.verts[ix.y], s);
    const Vtx c = project_vertex(P, m.verts[ix.z], s);
    const long long px = 256LL * i, py = 256LL * j;
    const long long w0 = edge_fn(b.U, b.V, c.U, c.V, px, py);
    const long long w1 = edge_fn(c.U, c.V, a.U, a.V, px, py);
    const long long w2 = edge_fn(a.U, a.V, b.U, b.V, px, py);
    const double t0 = (double)w0 * a.iz, t1 = (double)w1 * b.iz, t2 = (double)w2 * c.iz;
    const double sum = (t0 + t1) + t2;
    const uint32_t ca = m.vrgb[ix.x], cb = m.vrgb[ix.y], cc = m.vrgb[ix.z];
    uint32_t out = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const double c0 = (double)((ca >> (8 * ch)) & 255u);
        const double c1 = (double)((cb >> (8 * ch)) & 255u);
        const double c2 = (double)((cc >> (8 * ch)) & 255u);
        double v = rint(((t0 * c0 + t1 * c1) + t2 * c2) / sum);
        v = v < 0.0 ? 0.0 : (v > 255.0 ? 255.0 : v);
        out |= (uint32_t)v << (8 * ch);
    }
    return out;
}

// ------------------------------------------------------------------ colour

__device__ __forceinline__ float lab_f(float t)
{
    const float e = 216.0f / 24389.0f;
    const float k = 841.0f / 108.0f;
    return t > e ? cbrtf(t) : t * k + 4.0f / 29.0f;
}

__device__ __forceinline__ float4 srgb_to_lab(uint32_t c)
{
    const float r = c_lin[c & 255u], g = c_lin[(c >> 8) & 255u], b = c_lin[(c >> 16) & 255u];
    const float X = (0.4124f * r + 0.3576f * g) + 0.1805f * b;
    const float Y = (0.2126f * r + 0.7152f * g) + 0.0722f * b;
    const float Z = (0.0193f * r + 0.1192f * g) + 0.9505f * b;
    const float Xn = (0.4124f + 0.3576f) + 0.1805f;
    const float Yn = (0.2126f + 0.7152f) + 0.0722f;
    const float Zn = (0.0193f + 0.1192f) + 0.9505f;
    const float fx = lab_f(X / Xn), fy = lab_f(Y / Yn), fz = lab_f(Z / Zn);
    return make_float4(116.0f * fy - 16.0f, 500.0f * (fx - fy), 200.0f * (fy - fz), 0.0f);
}

// CIEDE2000 (kL = kC = kH = 1), binary32; x is the point, y its match.
__device__ float ciede2000(float4 x, float4 y)
{
    const float D2R = 0.017453292519943295f, R2D = 57.29577951308232f;
    const float P25 = 6103515625.0f;
    const float L1 = x.x, a1 = x.y, b1 = x.z;
    const float L2 = y.x, a2 = y.y, b2 = y.z;
    const float C1 = sqrtf(a1 * a1 + b1 * b1), C2 = sqrtf(a2 * a2 + b2 * b2);
    const float Cm = (C1 + C2) * 0.5f;
    const float Cm2 = Cm * Cm;
    const float Cm7 = ((Cm2 * Cm2) * Cm2) * Cm;
    const float G = 0.5f * (1.0f - sqrtf(Cm7 / (Cm7 + P25)));
    const float a1p = (1.0f + G) * a1, a2p = (1.0f + G) * a2;
    const float C1p = sqrtf(a1p * a1p + b1 * b1), C2p = sqrtf(a2p * a2p + b2 * b2);
    float h1p = (a1p == 0.0f && b1 == 0.0f) ? 0.0f : atan2f(b1, a1p) * R2D;
    float h2p = (a2p == 0.0f && b2 == 0.0f) ? 0.0f : atan2f(b2, a2p) * R2D;
    if (h1p < 0.0f) h1p += 360.0f;
    if (h2p < 0.0f) h2p += 360.0f;
    const float dLp = L2 - L1;
    const float dCp = C2p - C1p;
    const float CC = C1p * C2p;
    float dhp;
    if (CC == 0.0f) dhp = 0.0f;
    else if (fabsf(h2p - h1p) <= 180.0f) dhp = h2p - h1p;
    else if (h2p - h1p > 180.0f) dhp = h2p - h1p - 360.0f;
    else dhp = h2p - h1p + 360.0f;
    const float dHp = 2.0f * sqrtf(CC) * sinf(dhp * D2R * 0.5f);
    const float Lmp = (L1 + L2) * 0.5f;
    const float Cmp = (C1p + C2p) * 0.5f;
    float hmp;
    if (CC == 0.0f) hmp = h1p + h2p;
    else if (fabsf(h1p - h2p) <= 180.0f) hmp = (h1p + h2p) * 0.5f;
    else if (h1p + h2p < 360.0f) hmp = (h1p + h2p + 360.0f) * 0.5f;
    else hmp = (h1p + h2p - 360.0f) * 0.5f;
    const float T = 1.0f - 0.17f * cosf((hmp - 30.0f) * D2R) + 0.24f * cosf(2.0f * hmp * D2R)
                    + 0.32f * cosf((3.0f * hmp + 6.0f) * D2R) - 0.20f * cosf((4.0f * hmp - 63.0f) * D2R);
    const float hq = (hmp - 275.0f) / 25.0f;
    const float dth = 30.0f * expf(-(hq * hq));
    const float Cmp2 = Cmp * Cmp;
    const float Cmp7 = ((Cmp2 * Cmp2) * Cmp2) * Cmp;
    const float RC = 2.0f * sqrtf(Cmp7 / (Cmp7 + P25));
    const float Lm50 = (Lmp - 50.0f) * (Lmp - 50.0f);
    const float SL = 1.0f + 0.015f * Lm50 / sqrtf(20.0f + Lm50);
    const float SC = 1.0f + 0.045f * Cmp;
    const float SH = 1.0f + 0.015f * Cmp * T;
    const float RT = -sinf(2.0f * dth * D2R) * RC;
    const float tL = dLp / SL, tC = dCp / SC, tH = dHp / SH;
    return sqrtf(tL * tL + tC * tC + tH * tH + RT * tC * tH);
}

// ------------------------------------------------------------------ search

// Largest pixel offset along one axis between a point at lateral offset
// `lat` mm and depth `z` mm and any point within `dl` mm of it:
// f dl sqrt(lat^2 + z^2) / (z (z - dl)), plus one pixel of slack.
__device__ __forceinline__ int window_half(float f, float lat, float z, float dl, int limit)
{
    if (!(z > dl + 1.0f)) return limit;
    const float bnd = f * dl * sqrtf(lat * lat + z * z) / (z * (z - dl));
    if (!(bnd < (float)limit)) return limit;
    return (int)bnd + 1;
}

// Wave-cooperative window scans.  The caller's whole wave works on one
// point: each iteration covers one 8x8 block of the window, lane l taking
// pixel (l & 7, l >> 3) of the block; blocks whose depth range cannot hold a
// point within delta are skipped for the whole wave.

// Back-projection factors 16 (i - cx) / fx and 16 (j - cy) / fy, computed
// with the same correctly rounded binary64 operations as the per-column
// tables, so that no table load sits on the critical path.
__device__ __forceinline__ double kx_of(const SceneDev &s, int i)
{
    return (((double)i - (double)s.cx) * 16.0) / (double)s.fx;
}
__device__ __forceinline__ double ky_of(const SceneDev &s, int j)
{
    return (((double)j - (double)s.cy) * 16.0) / (double)s.fy;
}

// Mark, in the "explained" bitmap, every observed point within delta of the
// rendered point (i, j, d): the J_o side of Eq. 3 for this point.  The depth
// loads of four window blocks are issued before any of them is used.
template <bool G>
__device__ void wave_mark_neighbours(const SceneDev &s, int i, int j, int d, uint32_t *bm, int bx0, int by0,
                                     int bmw, int bmh, int lane)
{
    const int X = (int)rint(s.kx[i] * (double)d);
    const int Y = (int)rint(s.ky[j] * (double)d);
    const float dl = s.delta + 0.25f;
    const int wu = window_half(s.fx, (float)X * 0.0625f, (float)d, dl, s.W);
    const int wv = window_half(s.fy, (float)Y * 0.0625f, (float)d, dl, s.H);
    const int i0 = max(i - wu, 0), i1 = min(i + wu, s.W - 1);
    const int j0 = max(j - wv, 0), j1 = min(j + wv, s.H - 1);
    const int Z = 16 * d;
    const int bxa = i0 >> 3, bya = j0 >> 3;
    const int nbw = (i1 >> 3) - bxa + 1;
    const int nb = nbw * ((j1 >> 3) - bya + 1);
    for (int b0 = 0; b0 < nb; b0 += 4) {
        int dp[4], px[4], py[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + u;
            const int by = bya + b / nbw, bx = bxa + b % nbw;
            px[u] = (bx << 3) + (lane & 7);
            py[u] = (by << 3) + (lane >> 3);
            const bool in = b < nb && px[u] >= i0 && px[u] <= i1 && py[u] >= j0 && py[u] <= j1;
            dp[u] = in ? (int)s.depth[py[u] * s.W + px[u]] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int dz = 16 * dp[u] - Z;
            if (dp[u] == 0 || dz > s.dq || dz < -s.dq) continue;
            const int dx = (int)rint(kx_of(s, px[u]) * (double)dp[u]) - X;
            const int dy = (int)rint(ky_of(s, py[u]) * (double)dp[u]) - Y;
            if (dx > s.dq || dx < -s.dq || dy > s.dq || dy < -s.dq) continue;
            if (dx * dx + dy * dy + dz * dz > s.dq2) continue;
            const int bxr = px[u] - bx0, byr = py[u] - by0;
            if (bxr < 0 || bxr >= bmw || byr < 0 || byr >= bmh) continue;  // never taken: window <= (wtx, wty)
            const int bit = byr * bmw + bxr;
            if constexpr (G)
                __hip_atomic_fetch_or(bm + (bit >> 5), 1u << (bit & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                atomicOr(bm + (bit >> 5), 1u << (bit & 31));
        }
    }
}

// Nearest rendered point of the tile within delta of observed point
// (i, j, dp, X, Y): the smallest (squared distance, tile index), returned to
// every lane; ~0 if none.
template <bool G>
__device__ unsigned long long wave_nearest_rendered(const SceneDev &s, const uint32_t *tile, const uint32_t *rbmin,
                                                    const uint32_t *rbmax, const PoseInfo &in, int nbx, int i,
                                                    int j, int dp, int X, int Y, int lane)
{
    const float dl = s.delta + 0.25f;
    const int wu = window_half(s.fx, (float)X * 0.0625f, (float)dp, dl, s.W);
    const int wv = window_half(s.fy, (float)Y * 0.0625f, (float)dp, dl, s.H);
    const int i0 = max(i - wu, in.tx0) - in.tx0, i1 = min(i + wu, in.tx0 + in.tw - 1) - in.tx0;
    const int j0 = max(j - wv, in.ty0) - in.ty0, j1 = min(j + wv, in.ty0 + in.th - 1) - in.ty0;
    const int dlo = dp - s.dzmm, dhi = dp + s.dzmm;
    const int Z = 16 * dp;
    unsigned long long best = ~0ULL;
    if (i0 <= i1 && j0 <= j1) {
        for (int by = j0 >> 3; by <= (j1 >> 3); ++by) {
            for (int bx = i0 >> 3; bx <= (i1 >> 3); ++bx) {
                const int b = by * nbx + bx;
                if ((int)tld<G>(rbmax + b) < dlo || (int)tld<G>(rbmin + b) > dhi) continue;
                const int tx = (bx << 3) + (lane & 7), ty = (by << 3) + (lane >> 3);
                if (tx < i0 || tx > i1 || ty < j0 || ty > j1) continue;
                const int k = ty * in.tw + tx;
                const uint32_t key = tld<G>(tile + k);
                if (key == kEmptyKey) continue;
                const int dr = (int)(key >> 16);
                const int dz = Z - 16 * dr;
                if (dz > s.dq || dz < -s.dq) continue;
                const int dx = X - (int)rint(kx_of(s, in.tx0 + tx) * (double)dr);
                const int dy = Y - (int)rint(ky_of(s, in.ty0 + ty) * (double)dr);
                if (dx > s.dq || dx < -s.dq || dy > s.dq || dy < -s.dq) continue;
                const int d2 = dx * dx + dy * dy + dz * dz;
                if (d2 > s.dq2) continue;
                const unsigned long long c = ((unsigned long long)d2 << 32) | (uint32_t)k;
                best = c < best ? c : best;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
    }
    return best;
}

// Is observed point (X, Y, Z in 1/16 mm) inside the object's AABB at pose P,
// inflated by delta?  q = R^T (p - t), tested in binary64.
__device__ __forceinline__ bool in_volume(const MeshDev &m, const float *P, int X, int Y, int dp, double dl)
{
    const double e0 = (double)X / 16.0 - (double)P[3];
    const double e1 = (double)Y / 16.0 - (double)P[7];
    const double e2 = (double)dp - (double)P[11];
    const double q0 = ((double)P[0] * e0 + (double)P[4] * e1) + (double)P[8] * e2;
    const double q1 = ((double)P[1] * e0 + (double)P[5] * e1) + (double)P[9] * e2;
    const double q2 = ((double)P[2] * e0 + (double)P[6] * e1) + (double)P[10] * e2;
    return ((double)m.lo[0] - dl <= q0) && (q0 <= (double)m.hi[0] + dl) && ((double)m.lo[1] - dl <= q1)
           && (q1 <= (double)m.hi[1] + dl) && ((double)m.lo[2] - dl <= q2) && (q2 <= (double)m.hi[2] + dl);
}

__device__ __forceinline__ int wave_popc(bool pred)
{
    return __popcll(__ballot(pred));
}

// ------------------------------------------------------------------ per pose

template <int BLOCK, bool G, bool RGB>
__device__ void score_pose(const SceneDev &s, const MeshDev &m, const Work &w, int p, uint32_t *tile,
                           uint32_t *rbmin, uint32_t *rbmax, uint32_t *bm, int *cnt, int *queue, int *qn)
{
    constexpr int NW = BLOCK / 64;
    const int wave = threadIdx.x >> 6;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const PoseInfo in = w.info[p];
    float P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = w.poses[12 * (size_t)p + k];
    const int tpx = in.tw * in.th;
    const int nbx = (in.tw + 7) >> 3, nby = (in.th + 7) >> 3;
    const bool mark = (s.flags & 2u) != 0;
    const bool label_mode = (s.flags & (3u << 4)) == (2u << 4);

    for (int k = tid; k < tpx; k += BLOCK) tst<G>(tile + k, kEmptyKey);
    for (int k = tid; k < nbx * nby; k += BLOCK) {
        tst<G>(rbmin + k, 0xFFFFu);
        tst<G>(rbmax + k, 0u);
    }
    // explained-bitmap region: the tile dilated by the scene's neighbour window
    const int bx0 = in.tx0 - s.wtx, by0 = in.ty0 - s.wty;
    const int bmw = in.tw + 2 * s.wtx, bmh = in.th + 2 * s.wty;
    const int bmwords = (bmw * bmh + 31) >> 5;
    for (int k = tid; k < bmwords; k += BLOCK) tst<G>(bm + k, 0u);
    if (tid < 4) cnt[tid] = 0;
    __syncthreads();

    // 1. raster
    if (tpx > 0) {
        for (int t0 = 0; t0 < m.nt; t0 += BLOCK) {
            const int t = t0 + tid;
            if (t < m.nt) raster_triangle<G>(s, m, P, t, in.tx0, in.ty0, in.tw, in.th, tile);
        }
    }
    __syncthreads();

    // 2. resolve: occluders and stride
    int cL = 0;
    for (int k0 = 0; k0 < tpx; k0 += BLOCK) {
        const int k = k0 + tid;
        bool keep = false;
        if (k < tpx) {
            const uint32_t key = tld<G>(tile + k);
            if (key != kEmptyKey) {
                const int ty = k / in.tw, tx = k - ty * in.tw;
                const int i = in.tx0 + tx, j = in.ty0 + ty;
                const int d = (int)(key >> 16);
                keep = (i % s.stride == 0) && (j % s.stride == 0);
                if (keep && mark) {
                    const int pix = j * s.W + i;
                    const int dob = s.depth[pix];
                    if (dob > 0 && 16 * dob + s.dq < 16 * d) {
                        if (!(label_mode && s.labels) || s.labels[pix] != w.label) keep = false;
                    }
                }
                if (!keep) {
                    tst<G>(tile + k, kEmptyKey);
                } else {
                    const int b = (ty >> 3) * nbx + (tx >> 3);
                    tmin<G>(rbmin + b, (uint32_t)d);
                    tmax<G>(rbmax + b, (uint32_t)d);
                }
            }
        }
        cL += wave_popc(keep);
    }
    __syncthreads();

    // 3. J_r: nearest observed neighbour from the scene table.  The inliers
    //    of each chunk go to a workgroup queue, and every wave takes queue
    //    items in turn to mark their observed neighbours for J_o.
    int cR = 0;
    for (int k0 = 0; k0 < tpx; k0 += BLOCK) {
        const int k = k0 + tid;
        if (tid == 0) *qn = 0;
        __syncthreads();
        bool valid = false;
        int i = 0, j = 0, nn = -1;
        uint32_t key = kEmptyKey;
        if (k < tpx) {
            key = tld<G>(tile + k);
            if (key != kEmptyKey) {
                const int ty = k / in.tw, tx = k - ty * in.tw;
                i = in.tx0 + tx;
                j = in.ty0 + ty;
                valid = true;
                const int2 th = s.thdr[j * s.W + i];
                const int e = (int)(key >> 16) - (th.y & 0xFFFF);
                if (e >= 0 && e < (int)((uint32_t)th.y >> 16)) nn = s.tnn[th.x + e];
                if (nn >= 0) queue[atomicAdd(qn, 1)] = k;
            }
        }
        __syncthreads();
        const int nq = *qn;
        for (int t = wave; t < nq; t += NW) {
            const int kk = queue[t];
            const int ty = kk / in.tw, tx = kk - ty * in.tw;
            const int dd = (int)(tld<G>(tile + kk) >> 16);
            wave_mark_neighbours<G>(s, in.tx0 + tx, in.ty0 + ty, dd, bm, bx0, by0, bmw, bmh, lane);
        }
        bool out = valid && nn < 0;
        if (RGB && nn >= 0) {
            const float4 lr = srgb_to_lab(triangle_colour(s, m, P, (int)(key & 0xFFFFu), i, j));
            out = ciede2000(lr, s.olab[nn]) > s.tau;
        }
        cR += wave_popc(out);
        __syncthreads();
    }

    // 4. J_o: observed points in V(O); explained iff marked.  In RGB mode the
    //    explained points of each chunk are queued and the waves find their
    //    nearest rendered points; the result replaces the queue entry.
    int cQ = 0, cO = 0;
    const int vpx = in.vw * in.vh;
    const double dl = (double)s.delta;
    for (int k0 = 0; k0 < vpx; k0 += BLOCK) {
        const int k = k0 + tid;
        if (RGB) {
            if (tid == 0) *qn = 0;
            __syncthreads();
        }
        bool inq = false, expl = false;
        int pix = 0, slot = -1;
        if (k < vpx) {
            const int vy = k / in.vw, vx = k - vy * in.vw;
            const int i = in.vx0 + vx, j = in.vy0 + vy;
            pix = j * s.W + i;
            const int dp = s.depth[pix];
            if (dp > 0) {
                const int2 q = s.oxy[pix];
                inq = label_mode ? (s.labels[pix] == w.label) : in_volume(m, P, q.x, q.y, dp, dl);
                const int bxr = i - bx0, byr = j - by0;
                if (inq && bxr >= 0 && bxr < bmw && byr >= 0 && byr < bmh) {
                    const int bit = byr * bmw + bxr;
                    expl = (tld<G>(bm + (bit >> 5)) >> (bit & 31)) & 1u;
                }
                if (RGB && expl) {
                    slot = atomicAdd(qn, 1);
                    queue[slot] = pix;
                }
            }
        }
        bool out = inq && !expl;
        if (RGB) {
            __syncthreads();
            const int nq = *qn;
            for (int t = wave; t < nq; t += NW) {
                const int qp = queue[t];
                const int qj = qp / s.W, qi = qp - qj * s.W;
                const int dp = s.depth[qp];
                const int2 q = s.oxy[qp];
                const unsigned long long r =
                    wave_nearest_rendered<G>(s, tile, rbmin, rbmax, in, nbx, qi, qj, dp, q.x, q.y, lane);
                if (lane == 0) queue[t] = r == ~0ULL ? -1 : (int)(r & 0xFFFFFFFFu);
            }
            __syncthreads();
            if (slot >= 0) {
                const int kr = queue[slot];
                if (kr >= 0) {
                    const uint32_t key = tld<G>(tile + kr);
                    const int ty = kr / in.tw, tx = kr - ty * in.tw;
                    const float4 lr =
                        srgb_to_lab(triangle_colour(s, m, P, (int)(key & 0xFFFFu), in.tx0 + tx, in.ty0 + ty));
                    out = ciede2000(s.olab[pix], lr) > s.tau;
                }
            }
            __syncthreads();
        }
        cQ += wave_popc(inq);
        cO += wave_popc(out);
    }

    if (lane == 0) {
        atomicAdd(&cnt[0], cR);
        atomicAdd(&cnt[1], cO);
        atomicAdd(&cnt[2], cL);
        atomicAdd(&cnt[3], cQ);
    }
    __syncthreads();
    if (tid == 0) {
        w.jr[p] = cnt[0];
        w.jo[p] = cnt[1];
        if (w.nr) w.nr[p] = cnt[2];
        if (w.nq) w.nq[p] = cnt[3];
    }
    __syncthreads();
}

template <int BLOCK, bool G, bool RGB>
__global__ __launch_bounds__(BLOCK) void score_kernel(SceneDev s, MeshDev m, Work w, int cls, int cap, int nbcap)
{
    extern __shared__ uint32_t smem[];
    __shared__ int cnt[4];
    __shared__ int queue[BLOCK];
    __shared__ int qn;
    const int count = w.counts[cls];
    uint32_t *tile, *rbmin, *rbmax, *bm;
    if constexpr (G) {
        tile = w.gscratch + (size_t)blockIdx.x * w.gscratch_stride;
        rbmin = tile + (size_t)s.W * s.H;
        rbmax = rbmin + (size_t)s.bw * s.bh;
        bm = rbmax + (size_t)s.bw * s.bh;
    } else {
        tile = smem;
        rbmin = smem + cap;
        rbmax = rbmin + nbcap;
        bm = rbmax + nbcap;
    }
    for (int it = blockIdx.x; it < count; it += gridDim.x) {
        const int p = w.lists[cls * w.n + it];
        score_pose<BLOCK, G, RGB>(s, m, w, p, tile, rbmin, rbmax, bm, cnt, queue, &qn);
    }
}

// ------------------------------------------------------------------ setup

__device__ __forceinline__ void project_box(const float *P, const float lo[3], const float hi[3], double pad,
                                            const SceneDev &s, double *umin, double *umax, double *vmin,
                                            double *vmax, double *zmin, double *zmax)
{
    *umin = *vmin = *zmin = 1e300;
    *umax = *vmax = *zmax = -1e300;
    for (int c = 0; c < 8; ++c) {
        const double x = (c & 1) ? (double)hi[0] + pad : (double)lo[0] - pad;
        const double y = (c & 2) ? (double)hi[1] + pad : (double)lo[1] - pad;
        const double z = (c & 4) ? (double)hi[2] + pad : (double)lo[2] - pad;
        const double X = (((double)P[0] * x + (double)P[1] * y) + (double)P[2] * z) + (double)P[3];
        const double Y = (((double)P[4] * x + (double)P[5] * y) + (double)P[6] * z) + (double)P[7];
        const double Z = (((double)P[8] * x + (double)P[9] * y) + (double)P[10] * z) + (double)P[11];
        *zmin = fmin(*zmin, Z);
        *zmax = fmax(*zmax, Z);
        if (Z > 0.0) {
            const double u = (double)s.fx * X / Z + (double)s.cx;
            const double v = (double)s.fy * Y / Z + (double)s.cy;
            *umin = fmin(*umin, u);
            *umax = fmax(*umax, u);
            *vmin = fmin(*vmin, v);
            *vmax = fmax(*vmax, v);
        }
    }
}

__device__ __forceinline__ void clip_box(double umin, double umax, double vmin, double vmax, int W, int H, int *x0,
                                         int *y0, int *w, int *h)
{
    const double a = fmax(floor(umin) - 1.0, 0.0), b = fmin(ceil(umax) + 1.0, (double)(W - 1));
    const double c = fmax(floor(vmin) - 1.0, 0.0), d = fmin(ceil(vmax) + 1.0, (double)(H - 1));
    if (a > b || c > d) {
        *x0 = *y0 = *w = *h = 0;
        return;
    }
    *x0 = (int)a;
    *y0 = (int)c;
    *w = (int)b - (int)a + 1;
    *h = (int)d - (int)c + 1;
}

__global__ void zero_counts_kernel(int *counts)
{
    if (threadIdx.x < kNumClasses) counts[threadIdx.x] = 0;
}

__global__ void setup_kernel(SceneDev s, MeshDev m, Work w)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= w.n) return;
    float P[12];
    for (int k = 0; k < 12; ++k) P[k] = w.poses[12 * (size_t)p + k];
    PoseInfo in;
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
        in.vx0 = w.vbox_label[0];
        in.vy0 = w.vbox_label[1];
        in.vw = w.vbox_label[2];
        in.vh = w.vbox_label[3];
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
    w.info[p] = in;
    const int px = in.tw * in.th;
    const int cls = px <= w.cap_small ? 0 : (px <= w.cap_large ? 1 : 2);
    const int slot = atomicAdd(&w.counts[cls], 1);
    w.lists[cls * w.n + slot] = p;
}

// ------------------------------------------------------------------ scene prep

__global__ void scene_points_kernel(SceneDev s, const uint8_t *rgb, int2 *oxy, float4 *olab)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.W * s.H) return;
    const int j = k / s.W, i = k - j * s.W;
    const int d = s.depth[k];
    int2 q = make_int2(0, 0);
    if (d > 0) {
        q.x = (int)rint(s.kx[i] * (double)d);
        q.y = (int)rint(s.ky[j] * (double)d);
    }
    oxy[k] = q;
    if (olab) {
        const uint32_t c = (uint32_t)rgb[3 * (size_t)k] | ((uint32_t)rgb[3 * (size_t)k + 1] << 8)
                           | ((uint32_t)rgb[3 * (size_t)k + 2] << 16);
        olab[k] = srgb_to_lab(c);
    }
}

__global__ void scene_blocks_kernel(SceneDev s, uint32_t *oblk)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= s.bw * s.bh) return;
    const int by = b / s.bw, bx = b - by * s.bw;
    int mn = 0xFFFF, mx = 0;
    for (int j = by * 8; j < min(by * 8 + 8, s.H); ++j)
        for (int i = bx * 8; i < min(bx * 8 + 8, s.W); ++i) {
            const int d = s.depth[j * s.W + i];
            if (d == 0) continue;
            mn = min(mn, d);
            mx = max(mx, d);
        }
    oblk[b] = (uint32_t)mn | ((uint32_t)mx << 16);
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

// Exclusive scan of the per-pixel entry counts into thdr[].x (one block).
__global__ __launch_bounds__(1024) void table_scan_kernel(int N, int2 *thdr, long long *total)
{
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int chunk = (N + 1023) / 1024;
    const int a = t * chunk, b = min(a + chunk, N);
    long long sum = 0;
    for (int k = a; k < b; ++k) sum += (long long)((uint32_t)thdr[k].y >> 16);
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        long long run = 0;
        for (int k = 0; k < 1024; ++k) {
            const long long v = part[k];
            part[k] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    long long run = part[t];
    for (int k = a; k < b; ++k) {
        const int n = (int)((uint32_t)thdr[k].y >> 16);
        thdr[k].x = (int)run;
        run += n;
    }
}

// One wave per pixel: each lane takes one depth of the pixel's range and
// finds the nearest observed point within delta (ties: lower pixel index),
// scanning the window of the chunk's smallest depth (the widest one) with
// wave-uniform loads of the observed data.
__global__ __launch_bounds__(256) void table_fill_kernel(SceneDev s, int32_t *tnn)
{
    const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (a >= s.W * s.H) return;
    const int2 th = s.thdr[a];
    const int lo = th.y & 0xFFFF, n = (int)((uint32_t)th.y >> 16);
    if (n == 0) return;
    const int j = a / s.W, i = a - j * s.W;
    const double kxi = s.kx[i], kyj = s.ky[j];
    const float dl = s.delta + 0.25f;
    for (int e0 = 0; e0 < n; e0 += 64) {
        const int e = e0 + lane;
        const int d = lo + min(e, n - 1);
        const int X = (int)rint(kxi * (double)d);
        const int Y = (int)rint(kyj * (double)d);
        const int Z = 16 * d;
        const int dmin = lo + e0, dmax = lo + min(e0 + 63, n - 1);
        const int Xmin = (int)rint(kxi * (double)dmin), Ymin = (int)rint(kyj * (double)dmin);
        const int wu = window_half(s.fx, (float)Xmin * 0.0625f, (float)dmin, dl, s.W);
        const int wv = window_half(s.fy, (float)Ymin * 0.0625f, (float)dmin, dl, s.H);
        const int i0 = max(i - wu, 0), i1 = min(i + wu, s.W - 1);
        const int j0 = max(j - wv, 0), j1 = min(j + wv, s.H - 1);
        const int dlo = dmin - s.dzmm, dhi = dmax + s.dzmm;
        unsigned long long best = ~0ULL;
        for (int by = j0 >> 3; by <= (j1 >> 3); ++by) {
            for (int bx = i0 >> 3; bx <= (i1 >> 3); ++bx) {
                const uint32_t blk = s.oblk[by * s.bw + bx];
                if ((int)(blk >> 16) < dlo || (int)(blk & 0xFFFFu) > dhi) continue;
                const int ja = max(by << 3, j0), jb = min((by << 3) + 7, j1);
                const int ia = max(bx << 3, i0), ib = min((bx << 3) + 7, i1);
                for (int jj = ja; jj <= jb; ++jj) {
                    for (int ii = ia; ii <= ib; ++ii) {
                        const int pix = jj * s.W + ii;
                        const int dp = s.depth[pix];
                        if (dp < dlo || dp > dhi || dp == 0) continue;
                        const int2 q = s.oxy[pix];
                        const int dz = 16 * dp - Z;
                        const int dx = q.x - X, dy = q.y - Y;
                        if (dz > s.dq || dz < -s.dq || dx > s.dq || dx < -s.dq || dy > s.dq || dy < -s.dq) continue;
                        const int d2 = dx * dx + dy * dy + dz * dz;
                        if (d2 > s.dq2) continue;
                        const unsigned long long key = ((unsigned long long)d2 << 32) | (uint32_t)pix;
                        best = key < best ? key : best;
                    }
                }
            }
        }
        if (e < n) tnn[th.x + e] = best == ~0ULL ? -1 : (int32_t)(best & 0xFFFFFFFFu);
    }
}

hipError_t launch_table_ranges(const SceneDev &s, uint32_t *tmp, int2 *thdr, long long *total, hipStream_t st)
{
    const int N = s.W * s.H;
    table_rows_kernel<<<(N + 255) / 256, 256, 0, st>>>(s, tmp);
    table_cols_kernel<<<(N + 255) / 256, 256, 0, st>>>(s, tmp, thdr);
    table_scan_kernel<<<1, 1024, 0, st>>>(N, thdr, total);
    return hipGetLastError();
}

hipError_t launch_table_fill(const SceneDev &s, int32_t *tnn, hipStream_t st)
{
    const int N = s.W * s.H;
    table_fill_kernel<<<(N + 3) / 4, 256, 0, st>>>(s, tnn);
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

// Minimum of J = jr + jo with the lowest index among ties; out2 = {idx, J}.
__global__ __launch_bounds__(1024) void argmin_kernel(const int32_t *jr, const int32_t *jo, int n, int32_t *out2)
{
    __shared__ unsigned long long red[16];
    unsigned long long best = ~0ULL;
    for (int k = threadIdx.x; k < n; k += 1024) {
        const unsigned long long key = ((unsigned long long)(uint32_t)(jr[k] + jo[k]) << 32) | (uint32_t)k;
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
            out2[0] = (int32_t)(best & 0xFFFFFFFFu);
            out2[1] = (int32_t)(best >> 32);
        }
    }
}

// ------------------------------------------------------------------ launchers

size_t lds_bytes_for(int cap, int W, int H, int wtx, int wty)
{
    return (size_t)cap * 4 + (size_t)nbcap_for(cap, W, H) * 8 + (size_t)bmcap_for(cap, W, H, wtx, wty) * 4;
}

hipError_t upload_colour_table(const float *lin256)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lin), lin256, 256 * sizeof(float));
}

hipError_t launch_scene_prep(const SceneDev &s, const uint8_t *rgb_dev, int2 *oxy, float4 *olab, uint32_t *oblk,
                             hipStream_t st)
{
    const int N = s.W * s.H;
    scene_points_kernel<<<(N + 255) / 256, 256, 0, st>>>(s, rgb_dev, oxy, olab);
    const int nb = s.bw * s.bh;
    scene_blocks_kernel<<<(nb + 255) / 256, 256, 0, st>>>(s, oblk);
    return hipGetLastError();
}

template <bool RGB>
static hipError_t launch_class_t(const SceneDev &s, const MeshDev &m, const Work &w, const LaunchCfg &c, int cls,
                                 hipStream_t st)
{
    if (cls == 0) {
        const size_t lds = lds_bytes_for(c.cap_small, s.W, s.H, s.wtx, s.wty);
        hipError_t e = hipFuncSetAttribute((const void *)score_kernel<512, false, RGB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        score_kernel<512, false, RGB><<<c.grid_small, 512, lds, st>>>(s, m, w, 0, c.cap_small,
                                                                      nbcap_for(c.cap_small, s.W, s.H));
    } else if (cls == 1) {
        const size_t lds = lds_bytes_for(c.cap_large, s.W, s.H, s.wtx, s.wty);
        hipError_t e = hipFuncSetAttribute((const void *)score_kernel<1024, false, RGB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        score_kernel<1024, false, RGB><<<c.grid_large, 1024, lds, st>>>(s, m, w, 1, c.cap_large,
                                                                        nbcap_for(c.cap_large, s.W, s.H));
    } else {
        score_kernel<256, true, RGB><<<c.grid_ovf, 256, 0, st>>>(s, m, w, 2, 0, 0);
    }
    return hipGetLastError();
}

hipError_t launch_setup(const SceneDev &s, const MeshDev &m, const Work &w, hipStream_t st)
{
    zero_counts_kernel<<<1, 64, 0, st>>>(w.counts);
    setup_kernel<<<(w.n + 255) / 256, 256, 0, st>>>(s, m, w);
    return hipGetLastError();
}

hipError_t launch_score_class(const SceneDev &s, const MeshDev &m, const Work &w, const LaunchCfg &c, int cls,
                              hipStream_t st)
{
    return (s.flags & 1u) ? launch_class_t<true>(s, m, w, c, cls, st) : launch_class_t<false>(s, m, w, c, cls, st);
}

hipError_t launch_render(const SceneDev &s, const MeshDev &m, const float *poses, int n, uint32_t *keys,
                         uint16_t *depth, uint8_t *rgb, int32_t *tri, hipStream_t st)
{
    render_kernel<<<n, 256, 0, st>>>(s, m, poses, keys, depth, rgb, tri);
    return hipGetLastError();
}

hipError_t launch_argmin(const int32_t *jr, const int32_t *jo, int n, int32_t *out2, hipStream_t st)
{
    argmin_kernel<<<1, 1024, 0, st>>>(jr, jo, n, out2);
    return hipGetLastError();
}

}  // namespace perch
