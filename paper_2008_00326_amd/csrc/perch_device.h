// Device helpers shared by the gfx950 kernels: global loads, the rasterizer
// (Sec. IV-A "Parallel Rendering": binary64 transform and projection, 8
// sub-pixel bits, int64 edge functions with the top-left rule, binary64
// perspective depth, min-combined 32-bit (depth << 16 | triangle) keys),
// the projected box of a pose, the colour of a rendered pixel, CIELAB and
// CIEDE2000 (Eq. 4), the volume V(O) of Eq. 3, neighbour search windows,
// and small integer helpers.
#pragma once

#include "perch_internal.h"

#include <math.h>

namespace perch {

// Load through a global-address-space pointer: the scene, mesh and pose
// arrays are reached through descriptors in device memory, which the
// compiler would otherwise access with flat instructions.
#define PERCH_GLOBAL __attribute__((address_space(1)))
typedef int perch_v2i __attribute__((ext_vector_type(2)));
typedef int perch_v4i __attribute__((ext_vector_type(4)));
typedef float perch_v4f __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T gld(const T *p)
{
    return *(const PERCH_GLOBAL T *)p;
}
template <>
__device__ __forceinline__ int2 gld(const int2 *p)
{
    const perch_v2i v = *(const PERCH_GLOBAL perch_v2i *)p;
    return make_int2(v.x, v.y);
}
template <>
__device__ __forceinline__ int4 gld(const int4 *p)
{
    const perch_v4i v = *(const PERCH_GLOBAL perch_v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
template <>
__device__ __forceinline__ float4 gld(const float4 *p)
{
    const perch_v4f v = *(const PERCH_GLOBAL perch_v4f *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// Observed point (Xq, Yq, Zq) of scene pixel `pix`: a 12-byte load (the
// image's fourth word is padding, and a wider load would leave a dead
// destination register that the allocator reuses before the load lands,
// forcing a wait) at a 32-bit byte offset from the image base.
__device__ __forceinline__ int3 opt_at(const int4 *opt, uint32_t pix)
{
    typedef int v3i __attribute__((ext_vector_type(3)));
    const v3i v = *(const PERCH_GLOBAL v3i *)((const PERCH_GLOBAL char *)opt + pix * 16u);
    return make_int3(v.x, v.y, v.z);
}

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
// A projected vertex packed in 16 bytes (U, V, iz), for a per-pose cache in
// LDS; iz < 0 marks a vertex that takes part in no drawn triangle.
__device__ __forceinline__ int4 pack_vtx(const Vtx &v)
{
    const long long b = __double_as_longlong(v.ok ? v.iz : -1.0);
    return make_int4(v.U, v.V, (int)(uint32_t)b, (int)(uint32_t)(b >> 32));
}
__device__ __forceinline__ Vtx unpack_vtx(int4 q)
{
    Vtx v;
    v.U = q.x;
    v.V = q.y;
    v.iz = __longlong_as_double(((long long)(uint32_t)q.w << 32) | (uint32_t)q.z);
    v.ok = v.iz > 0.0;
    return v;
}

// Scan of a triangle's pixel box [i0, i1] x [j0, j1]: edge functions
// stepped incrementally in integer type E (exact either way; see
// raster_triangle for when 32 bits suffice), covered pixels' binary64
// perspective depth min-combined into the tile.
template <bool G, class E>
__device__ __forceinline__ void raster_box(const Vtx &a, const Vtx &b, const Vtx &c, double farea, int t, int i0,
                                           int i1, int j0, int j1, int tx0, int ty0, int tw, uint32_t *tile)
{
    const E px0 = (E)256 * i0, py0 = (E)256 * j0;
    E r0 = (E)(c.V - b.V) * (px0 - b.U) - (E)(c.U - b.U) * (py0 - b.V);
    E r1 = (E)(a.V - c.V) * (px0 - c.U) - (E)(a.U - c.U) * (py0 - c.V);
    E r2 = (E)(b.V - a.V) * (px0 - a.U) - (E)(b.U - a.U) * (py0 - a.V);
    const E sx0 = (E)256 * (c.V - b.V), sy0 = (E)-256 * (c.U - b.U);
    const E sx1 = (E)256 * (a.V - c.V), sy1 = (E)-256 * (a.U - c.U);
    const E sx2 = (E)256 * (b.V - a.V), sy2 = (E)-256 * (b.U - a.U);
    const E b0 = (E)edge_bias(b.U, b.V, c.U, c.V);
    const E b1 = (E)edge_bias(c.U, c.V, a.U, a.V);
    const E b2 = (E)edge_bias(a.U, a.V, b.U, b.V);
    for (int j = j0; j <= j1; ++j) {
        E w0 = r0, w1 = r1, w2 = r2;
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

// Rasterize triangle t into the tile covering pixels [tx0, tx0+tw) x [ty0, ty0+th).
// vcache, when given, holds every vertex projected at this pose.
template <bool G>
__device__ __forceinline__ void raster_triangle(const SceneDev &s, const MeshDev &m, const float *P,
                                                int t, int tx0, int ty0, int tw, int th,
                                                uint32_t *tile, const int4 *vcache = nullptr)
{
    const int4 ix = gld(m.tris + t);
    Vtx a, b, c;
    if (vcache) {
        a = unpack_vtx(vcache[ix.x]);
        b = unpack_vtx(vcache[ix.y]);
        c = unpack_vtx(vcache[ix.z]);
    } else {
        a = project_vertex(P, gld(m.verts + ix.x), s);
        b = project_vertex(P, gld(m.verts + ix.y), s);
        c = project_vertex(P, gld(m.verts + ix.z), s);
    }
    if (!(a.ok & b.ok & c.ok)) return;
    const long long area = edge_fn(a.U, a.V, b.U, b.V, c.U, c.V);
    if (area <= 0) return;
    const int minU = min(a.U, min(b.U, c.U)), maxU = max(a.U, max(b.U, c.U));
    const int minV = min(a.V, min(b.V, c.V)), maxV = max(a.V, max(b.V, c.V));
    const int i0 = max(-((-minU) >> 8), tx0), i1 = min(maxU >> 8, tx0 + tw - 1);
    const int j0 = max(-((-minV) >> 8), ty0), j1 = min(maxV >> 8, ty0 + th - 1);
    if (i0 > i1 || j0 > j1) return;
    // Every pixel sample the scan evaluates, one step past the box included,
    // lies within 256 sub-pixel units of the triangle's box, so each edge
    // function is bounded by 2 (du + 256)(dv + 256) for box extents du, dv:
    // below 2^31 when both are under 2^15 - 256, the common case.
    if (maxU - minU < 32512 && maxV - minV < 32512)
        raster_box<G, int>(a, b, c, (double)area, t, i0, i1, j0, j1, tx0, ty0, tw, tile);
    else
        raster_box<G, long long>(a, b, c, (double)area, t, i0, i1, j0, j1, tx0, ty0, tw, tile);
}

// ------------------------------------------------------------------ screen boxes

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

// sRGB8 -> linear, rounded from binary64; each translation unit that converts
// colours holds its own copy and fills it at initialisation
static __constant__ float c_lin[256];

// ------------------------------------------------------------------ colour of a pixel

// Perspective-correct vertex colour of triangle t at pixel (i, j), rounded to sRGB8.
__device__ uint32_t triangle_colour(const SceneDev &s, const MeshDev &m, const float *P, int t, int i, int j)
{
    if (t < 0 || t >= m.nt) return 0;
    const int4 ix = gld(m.tris + t);
    const Vtx a = project_vertex(P, gld(m.verts + ix.x), s);
    const Vtx b = project_vertex(P, gld(m.verts + ix.y), s);
    const Vtx c = project_vertex(P, gld(m.verts + ix.z), s);
    const long long px = 256LL * i, py = 256LL * j;
    const long long w0 = edge_fn(b.U, b.V, c.U, c.V, px, py);
    const long long w1 = edge_fn(c.U, c.V, a.U, a.V, px, py);
    const long long w2 = edge_fn(a.U, a.V, b.U, b.V, px, py);
    const double t0 = (double)w0 * a.iz, t1 = (double)w1 * b.iz, t2 = (double)w2 * c.iz;
    const double sum = (t0 + t1) + t2;
    const uint32_t ca = gld(m.vrgb + ix.x), cb = gld(m.vrgb + ix.y), cc = gld(m.vrgb + ix.z);
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
    // T from one sine and cosine of the mean hue: the multiple angles by
    // the double- and triple-angle formulas, the offsets (30, 6 and 63
    // degrees) by angle addition with constant sines and cosines
    float s1, c1;
    sincosf(hmp * D2R, &s1, &c1);
    const float c2 = c1 * c1 - s1 * s1, s2 = 2.0f * s1 * c1;
    const float c3 = c1 * (c2 - 2.0f * s1 * s1), s3 = s1 * (2.0f * c1 * c1 + c2);
    const float c4 = c2 * c2 - s2 * s2, s4 = 2.0f * s2 * c2;
    const float C30 = 0.8660254037844386f, S30 = 0.5f;
    const float C6 = 0.9945218953682733f, S6 = 0.10452846326765347f;
    const float C63 = 0.45399049973954675f, S63 = 0.8910065241883679f;
    const float T = 1.0f - 0.17f * (c1 * C30 + s1 * S30) + 0.24f * c2 + 0.32f * (c3 * C6 - s3 * S6)
                    - 0.20f * (c4 * C63 + s4 * S63);
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

// ------------------------------------------------------------------ volumes and search windows

// Is observed point (X, Y, Z in 1/16 mm) inside V(O) at pose P?  q = R^T (p - t)
// in binary64, tested against the object's AABB inflated by delta or, for
// the cylinder volume, against the cylinder about the object z axis through
// the centre of the AABB's xy extent, of radius the smaller xy half-extent
// plus delta, over the AABB's z range inflated by delta.
__device__ __forceinline__ bool in_volume(const MeshDev &m, const float *P, int X, int Y, int dp, double dl, bool cyl)
{
    const double e0 = (double)X / 16.0 - (double)P[3];
    const double e1 = (double)Y / 16.0 - (double)P[7];
    const double e2 = (double)dp - (double)P[11];
    const double q0 = ((double)P[0] * e0 + (double)P[4] * e1) + (double)P[8] * e2;
    const double q1 = ((double)P[1] * e0 + (double)P[5] * e1) + (double)P[9] * e2;
    const double q2 = ((double)P[2] * e0 + (double)P[6] * e1) + (double)P[10] * e2;
    const bool inz = ((double)m.lo[2] - dl <= q2) && (q2 <= (double)m.hi[2] + dl);
    if (cyl) {
        const double c0 = ((double)m.lo[0] + (double)m.hi[0]) / 2.0, c1 = ((double)m.lo[1] + (double)m.hi[1]) / 2.0;
        const double h0 = ((double)m.hi[0] - (double)m.lo[0]) / 2.0, h1 = ((double)m.hi[1] - (double)m.lo[1]) / 2.0;
        const double rho = (h0 < h1 ? h0 : h1) + dl;
        const double a = q0 - c0, b = q1 - c1;
        return (a * a + b * b <= rho * rho) && inz;
    }
    return ((double)m.lo[0] - dl <= q0) && (q0 <= (double)m.hi[0] + dl) && ((double)m.lo[1] - dl <= q1)
           && (q1 <= (double)m.hi[1] + dl) && inz;
}

// Largest pixel offset along one axis between a point on the ray of pixel
// column (row) i at depth z mm and any point within dl = delta + 1/4 mm of
// it: f dl sqrt(1 + ((i - c) / f)^2) / (z - dl) = a[i] / (z - dl), with
// `inv` = 1 / (z - dl).  Every point here is the back-projection of a pixel
// centre at an integer depth, rounded to 1/16 mm: two points within delta in
// those units lie within delta + 0.12 mm before rounding, and their pixel
// offset, an integer, is at most the bound's floor.  a[i] is rounded up; the
// factor covers the binary32 rounding of the quotient (a few ulps).
__device__ __forceinline__ int window_half(float a, float inv, int limit)
{
    const float bnd = a * inv * 1.000002f;
    if (!(bnd < (float)limit)) return limit;
    return (int)bnd;
}

// 1 / (z - dl) for window_half, or infinity when z is too close to the
// camera for a bound (window_half then returns its limit).
__device__ __forceinline__ float window_inv(int z, float dl)
{
    const float den = (float)z - dl;
    return den > 1.0f ? 1.0f / den : INFINITY;
}

// ------------------------------------------------------------------ integer helpers

// Row of entry q of a row-major window ww pixels wide: a binary32 estimate
// corrected to the exact quotient.
__device__ __forceinline__ int window_row(int q, int ww, float inv)
{
    int qy = (int)(((float)q + 0.5f) * inv);
    if (qy * ww > q) --qy;
    else if ((qy + 1) * ww <= q) ++qy;
    return qy;
}

// v_med3_i32 as a clamp (lo <= hi).
__device__ __forceinline__ int clamp_i32(int x, int lo, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// ------------------------------------------------------------------ voxel hash

// Bucket of voxel cell (cx, cy, cz): the spatial hash of Teschner et al.
// (2003), three large primes xor-combined, masked to 2^bits buckets.
__device__ __forceinline__ int cell_bucket(int cx, int cy, int cz, int bits)
{
    const uint32_t h = ((uint32_t)cx * 73856093u) ^ ((uint32_t)cy * 19349663u) ^ ((uint32_t)cz * 83492791u);
    return (int)(h & ((1u << bits) - 1u));
}

// Nearest observed point within delta of (X, Y, Z) (1/16 mm) through the
// scene's voxel hash: the cells are at least delta wide, so every neighbour
// lies in one of the 27 cells around the point's own.  Smallest (d^2,
// pixel index), or -1.  Cells that share a bucket make the scan visit
// extra points, which the distance test rejects; a bucket scanned twice
// changes no minimum.
__device__ __noinline__ int hash_nn(const SceneDev &s, int X, int Y, int Z)
{
    const int lim = s.dq + 1, dq2 = s.dq2;
    const int cx = X >> s.hshift, cy = Y >> s.hshift, cz = Z >> s.hshift;
    int best = dq2 + 1, nn = -1;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int b = cell_bucket(cx + dx, cy + dy, cz + dz, s.hbits);
                const int e = gld(s.hstart + b + 1);
                for (int k = gld(s.hstart + b); k < e; ++k) {
                    const int4 q = gld(s.hpts + k);
                    const int ox = clamp_i32(q.x - X, -lim, lim);
                    const int oy = clamp_i32(q.y - Y, -lim, lim);
                    const int oz = clamp_i32(q.z - Z, -lim, lim);
                    const int d2 = __mul24(ox, ox) + __mul24(oy, oy) + __mul24(oz, oz);
                    if (d2 < best || (d2 == best && q.w < nn)) {
                        best = d2;
                        nn = q.w;
                    }
                }
            }
    return nn;
}

}  // namespace perch
