// Device helpers shared by the gfx950 kernels: global loads, the rasterizer
// (Sec. IV-A "Parallel Rendering": binary64 transform and projection, 8
// sub-pixel bits, int64 edge functions with the top-left rule, binary64
// perspective depth, min-combined 32-bit (depth << 16 | triangle) keys),
// the projected box of a pose, and small integer helpers.
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

}  // namespace perch
