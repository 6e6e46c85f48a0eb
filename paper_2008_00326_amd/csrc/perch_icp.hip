// gfx950 kernels for the steps around pose scoring: ICP refinement of
// candidate poses (Sec. IV-A "Parallel M2M GICP"; point-to-point, as in the
// 3-DoF experiments of Sec. VI-A) and 6-DoF pose proposals (Sec. V-B).
// Geometry in binary64 without FMA contraction (built with
// -ffp-contract=off), as the oracle computes it.

#include "perch_device.h"

namespace perch {

// ------------------------------------------------------------------ ICP refinement

// Per-iteration ICP sums over the matched pairs (q, c), one component per
// lane: n, q (3), c (3), q q^T (9, row-major), q c^T (9, row-major).
constexpr int kIcpSums = 25;

__device__ __forceinline__ long long icp_pick(int a, long long x, long long y, long long z)
{
    return a == 0 ? x : (a == 1 ? y : z);
}

__device__ __forceinline__ long long icp_term(int j, int4 q, int4 c)
{
    if (j == 0) return 1;
    if (j < 4) return icp_pick(j - 1, q.x, q.y, q.z);
    if (j < 7) return icp_pick(j - 4, c.x, c.y, c.z);
    if (j < 16) return icp_pick((j - 7) / 3, q.x, q.y, q.z) * icp_pick((j - 7) % 3, q.x, q.y, q.z);
    return icp_pick((j - 16) / 3, q.x, q.y, q.z) * icp_pick((j - 16) % 3, c.x, c.y, c.z);
}

// Nearest observed point of q (1/16 mm) within rq, ties to the lower pixel
// index, or -1; with `labels`, only pixels carrying `label` count (label
// volumes: the object's segment is the target), and `box` (inside the
// image) holds every pixel that can count.  The whole wave searches, lanes
// over a pixel window that holds every candidate: an observed point at
// depth d (mm) with
// |Xq - qx| <= rq has rint(kx[i] d) in [qx - rq, qx + rq], so
// kx[i] d lies within half a unit of that range, for d in
// [(qz - rq) / 16, (qz + rq) / 16]; one pixel of margin on each side.
__device__ int icp_nn(const SceneDev &s, int4 q, int rq, int rq2, const int32_t *labels, int label, const int *box,
                      int lane)
{
    const int dlo = q.z - rq <= 16 ? 1 : (q.z - rq + 15) / 16;
    const int dhi = min(65534, (q.z + rq) / 16);
    if (q.z + rq < 16 || dlo > dhi) return -1;
    const double lo_d = (double)dlo, hi_d = (double)dhi;
    int b[4];
    const int qv[2] = {q.x, q.y};
    for (int ax = 0; ax < 2; ++ax) {
        const double f16 = (double)(ax == 0 ? s.fx : s.fy) / 16.0, c = (double)(ax == 0 ? s.cx : s.cy);
        const double lo = (double)(qv[ax] - rq) - 0.5, hi = (double)(qv[ax] + rq) + 0.5;
        const double a = c + f16 * fmin(lo / lo_d, lo / hi_d), z = c + f16 * fmax(hi / lo_d, hi / hi_d);
        b[2 * ax] = (int)floor(fmax(fmin(a, 1e8), -1e8)) - 1;
        b[2 * ax + 1] = (int)ceil(fmax(fmin(z, 1e8), -1e8)) + 1;
    }
    const int i0 = max(b[0], box[0]), i1 = min(b[1], box[2]), j0 = max(b[2], box[1]), j1 = min(b[3], box[3]);
    if (i0 > i1 || j0 > j1) return -1;
    const int ww = i1 - i0 + 1, n = ww * (j1 - j0 + 1);
    const float inv = 1.0f / (float)ww;
    const int lim = rq + 1;
    unsigned long long best = ~0ULL;
    for (int k0 = 0; k0 < n; k0 += 64) {
        const int k = k0 + lane;
        if (k < n) {
            const int r = window_row(k, ww, inv);
            const int pix = (j0 + r) * s.W + i0 + (k - r * ww);
            const int4 o = gld(s.opt + pix);
            const int dx = clamp_i32(o.x - q.x, -lim, lim);
            const int dy = clamp_i32(o.y - q.y, -lim, lim);
            const int dz = clamp_i32(o.z - q.z, -lim, lim);
            const int d2 = __mul24(dx, dx) + __mul24(dy, dy) + __mul24(dz, dz);
            if (d2 <= rq2 && (!labels || gld(labels + pix) == label)) {
                const unsigned long long key = ((unsigned long long)(uint32_t)d2 << 32) | (uint32_t)pix;
                best = key < best ? key : best;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o < best ? o : best;
    }
    return best == ~0ULL ? -1 : (int)(best & 0xFFFFFFFFu);
}

// One ICP update from the sums (n, q, c, q q^T, q c^T): the increment about
// the source centroid mq composed into (A, b), b in 1/16 mm.  3-DoF: the
// planar Procrustes rotation about the unit axis u and the centroid moved
// within the plane normal to u; 6-DoF: a Gauss-Newton step of the
// linearised rotation, (tr(S) I - S) w' = w, mapped to a rotation by the
// unit quaternion (1, w'/2) and the centroid moved onto mc.  Every step
// uses + - * / and sqrt only, left to right.  Returns 1 when the 6-DoF
// system is singular (nothing changes).
__device__ int icp_update(const long long *z, int dof, const double u[3], double *A, double *b)
{
    const double n = (double)z[0];
    double mq[3], mc[3], S[3][3], H[3][3];
    for (int a = 0; a < 3; ++a) {
        mq[a] = (double)z[1 + a] / n;
        mc[a] = (double)z[4 + a] / n;
    }
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            S[a][c] = (double)z[7 + 3 * a + c] - ((double)z[1 + a] * (double)z[1 + c]) / n;
            H[a][c] = (double)z[16 + 3 * a + c] - ((double)z[1 + a] * (double)z[4 + c]) / n;
        }
    const double w[3] = {H[1][2] - H[2][1], H[2][0] - H[0][2], H[0][1] - H[1][0]};
    double R[3][3], mp[3];
    if (dof == 3) {
        double Hu[3];
        for (int a = 0; a < 3; ++a) Hu[a] = (H[a][0] * u[0] + H[a][1] * u[1]) + H[a][2] * u[2];
        const double uHu = (u[0] * Hu[0] + u[1] * Hu[1]) + u[2] * Hu[2];
        const double Ap = ((H[0][0] + H[1][1]) + H[2][2]) - uHu;
        const double B = (u[0] * w[0] + u[1] * w[1]) + u[2] * w[2];
        const double h = sqrt(Ap * Ap + B * B);
        double co = 1.0, si = 0.0;
        if (h > 0.0) {
            co = Ap / h;
            si = B / h;
        }
        const double Kx[3][3] = {{0.0, -u[2], u[1]}, {u[2], 0.0, -u[0]}, {-u[1], u[0], 0.0}};
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) R[a][c] = ((a == c ? co : 0.0) + si * Kx[a][c]) + ((1.0 - co) * u[a]) * u[c];
        const double d[3] = {mc[0] - mq[0], mc[1] - mq[1], mc[2] - mq[2]};
        const double ud = (u[0] * d[0] + u[1] * d[1]) + u[2] * d[2];
        for (int a = 0; a < 3; ++a) mp[a] = mq[a] + (d[a] - ud * u[a]);
    } else {
        const double tr = (S[0][0] + S[1][1]) + S[2][2];
        double M[3][3];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) M[a][c] = (a == c ? tr : 0.0) - S[a][c];
        double adj[3][3];
        adj[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
        adj[0][1] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
        adj[0][2] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
        adj[1][0] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
        adj[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
        adj[1][2] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
        adj[2][0] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
        adj[2][1] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
        adj[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
        const double det = (M[0][0] * adj[0][0] + M[0][1] * adj[1][0]) + M[0][2] * adj[2][0];
        if (!(det > 0.0)) return 1;
        double h[3];
        for (int a = 0; a < 3; ++a) h[a] = (((adj[a][0] * w[0] + adj[a][1] * w[1]) + adj[a][2] * w[2]) / det) / 2.0;
        const double r = sqrt(1.0 + ((h[0] * h[0] + h[1] * h[1]) + h[2] * h[2]));
        const double qw = 1.0 / r, qx = h[0] / r, qy = h[1] / r, qz = h[2] / r;
        R[0][0] = 1.0 - 2.0 * (qy * qy + qz * qz);
        R[0][1] = 2.0 * (qx * qy - qz * qw);
        R[0][2] = 2.0 * (qx * qz + qy * qw);
        R[1][0] = 2.0 * (qx * qy + qz * qw);
        R[1][1] = 1.0 - 2.0 * (qx * qx + qz * qz);
        R[1][2] = 2.0 * (qy * qz - qx * qw);
        R[2][0] = 2.0 * (qx * qz - qy * qw);
        R[2][1] = 2.0 * (qy * qz + qx * qw);
        R[2][2] = 1.0 - 2.0 * (qx * qx + qy * qy);
        for (int a = 0; a < 3; ++a) mp[a] = mc[a];
    }
    double An[9], bn[3];
    const double e[3] = {b[0] - mq[0], b[1] - mq[1], b[2] - mq[2]};
    for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c) An[3 * a + c] = (R[a][0] * A[c] + R[a][1] * A[3 + c]) + R[a][2] * A[6 + c];
        bn[a] = ((R[a][0] * e[0] + R[a][1] * e[1]) + R[a][2] * e[2]) + mp[a];
    }
    for (int k = 0; k < 9; ++k) A[k] = An[k];
    for (int k = 0; k < 3; ++k) b[k] = bn[k];
    return 0;
}

__global__ void icp_zero_kernel(int *cursor)
{
    if (threadIdx.x == 0) cursor[threadIdx.x] = 0;
}

// ICP refinement (Sec. IV-A "Parallel M2M GICP"; point-to-point): one pose
// per work-group at a time, taken through a cursor.  The pose is rendered
// into the work-group's device tile, its rendered points (R minus C on the
// ICP stride grid) collected, then each iteration maps them by the current
// transform (rounded to 1/16 mm), stops when no mapped point moved, matches
// each to its nearest observed point within rho (one wave per point), sums
// the pairs exactly in int64 and updates the transform on one thread.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void icp_kernel(IcpArgs a)
{
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const SceneDev &s = a.s;
    const MeshDev &m = a.m;
    extern __shared__ uint32_t icp_lds[];
    __shared__ int s_pose, s_n, s_box[4], s_changed, s_stop;
    __shared__ long long s_red[NW][kIcpSums];
    __shared__ double s_A[9], s_b[3];
    uint32_t *tile = a.tiles + (size_t)blockIdx.x * s.W * s.H;
    int4 *src = a.pts + (size_t)blockIdx.x * 2 * a.pts_cap;
    int4 *qb = src + a.pts_cap;
    const bool mark = (s.flags & 2u) != 0;
    const bool label_mode = (s.flags & (3u << 4)) == (2u << 4);
    for (;;) {
        if (tid == 0) s_pose = atomicAdd(a.cursor, 1);
        __syncthreads();
        const int p = s_pose;
        if (p >= a.n) break;
        float P[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) P[k] = a.poses[12 * (size_t)p + k];
        if (tid == 0) {
            double umin, umax, vmin, vmax, zmin, zmax;
            int x0 = 0, y0 = 0, w = 0, h = 0;
            project_box(P, m.lo, m.hi, 0.0, s, &umin, &umax, &vmin, &vmax, &zmin, &zmax);
            if (zmin >= 100.0) {
                clip_box(umin, umax, vmin, vmax, s.W, s.H, &x0, &y0, &w, &h);
                // Nothing in reach: every rendered point lies on a pixel of the
                // tile at depth >= zmin - 1/2 (depths are rounded to whole mm),
                // and a match lies within rho + 1/4 mm of it (points are rounded
                // to 1/16 mm), so its pixel is within
                // f (rho + 1/4) sqrt(1 + t^2) / (zmin - 1/2 - rho - 1/4) of the
                // tile (t the tile's largest ray slope), plus one.  When that
                // grown tile misses the target box, no point can match: the
                // pose comes back unchanged, as the iteration would return it.
                const double rp = (double)a.rq / 16.0 + 0.25;
                const double zn = zmin - 0.5;
                if (w > 0 && zn - rp > 1.0) {
                    const double tx = fmax(fabs((double)x0 - (double)s.cx), fabs((double)(x0 + w - 1) - (double)s.cx)) / (double)s.fx;
                    const double ty = fmax(fabs((double)y0 - (double)s.cy), fabs((double)(y0 + h - 1) - (double)s.cy)) / (double)s.fy;
                    const double du = (double)s.fx * rp * sqrt(1.0 + tx * tx) / (zn - rp) + 1.0;
                    const double dv = (double)s.fy * rp * sqrt(1.0 + ty * ty) / (zn - rp) + 1.0;
                    if ((double)(x0 + w - 1) + du < (double)a.box[0] || (double)x0 - du > (double)a.box[2]
                        || (double)(y0 + h - 1) + dv < (double)a.box[1] || (double)y0 - dv > (double)a.box[3])
                        w = h = 0;
                }
            } else if (!(zmax < 99.999)) {
                w = s.W;
                h = s.H;
            }
            s_box[0] = x0;
            s_box[1] = y0;
            s_box[2] = w;
            s_box[3] = h;
            s_n = 0;
            for (int k = 0; k < 9; ++k) s_A[k] = (k % 4 == 0) ? 1.0 : 0.0;
            s_b[0] = s_b[1] = s_b[2] = 0.0;
        }
        __syncthreads();
        const int tx0 = s_box[0], ty0 = s_box[1], tw = s_box[2], th = s_box[3];
        const int tpx = tw * th;
        // the tile in LDS when it fits (then, with room to spare, every
        // vertex projected once for the pose), else in device memory
        const bool in_lds = tpx <= a.lds_words;
        const int tile_q = (tpx + 3) & ~3;
        const int4 *vcache = nullptr;
        if (in_lds) {
            for (int k = tid; k < tpx; k += BLOCK) icp_lds[k] = kEmptyKey;
            if (tpx > 0 && 4 * m.nv <= a.lds_words - tile_q) {
                int4 *vc = reinterpret_cast<int4 *>(icp_lds + tile_q);
                for (int v = tid; v < m.nv; v += BLOCK) vc[v] = pack_vtx(project_vertex(P, gld(m.verts + v), s));
                vcache = vc;
            }
        } else {
            for (int k = tid; k < tpx; k += BLOCK) tst<true>(tile + k, kEmptyKey);
        }
        __syncthreads();
        if (tpx > 0)
            for (int t0 = 0; t0 < m.nt; t0 += BLOCK)
                if (t0 + tid < m.nt) {
                    if (in_lds) raster_triangle<false>(s, m, P, t0 + tid, tx0, ty0, tw, th, icp_lds, vcache);
                    else raster_triangle<true>(s, m, P, t0 + tid, tx0, ty0, tw, th, tile);
                }
        __syncthreads();
        for (int k = tid; k < tpx; k += BLOCK) {
            const uint32_t key = in_lds ? icp_lds[k] : tld<true>(tile + k);
            if (key == kEmptyKey) continue;
            const int ty = k / tw, tx = k - ty * tw;
            const int i = tx0 + tx, j = ty0 + ty, d = (int)(key >> 16);
            if (i % a.stride != 0 || j % a.stride != 0) continue;
            const int pix = j * s.W + i;
            if (mark) {
                const int dob = gld(s.depth + pix);
                if (dob > 0 && 16 * dob + s.dq < 16 * d && (!(label_mode && s.labels) || s.labels[pix] != a.label))
                    continue;
            }
            const int slot = atomicAdd(&s_n, 1);
            src[slot] = make_int4((int)rint(gld(s.kx + i) * (double)d), (int)rint(gld(s.ky + j) * (double)d), 16 * d, 0);
        }
        __syncthreads();
        const int ns = s_n;
        double u[3] = {0.0, 0.0, 0.0};
        int iters = 0, matched = 0;
        if (tid == 0) {
            const double v[3] = {(double)P[2], (double)P[6], (double)P[10]};
            const double nrm = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
            for (int c = 0; c < 3; ++c) u[c] = v[c] / nrm;
        }
        for (int it = 0; it < a.iterations; ++it) {
            if (tid == 0) s_changed = 0;
            __syncthreads();
            bool ch = false;
            for (int t = tid; t < ns; t += BLOCK) {
                const int4 sp = src[t];
                int qv[3];
                for (int c = 0; c < 3; ++c) {
                    // beyond 2^28 units (16 km) nothing can match; the clamp keeps the search in int range
                    const double v = rint(((s_A[3 * c] * (double)sp.x + s_A[3 * c + 1] * (double)sp.y)
                                           + s_A[3 * c + 2] * (double)sp.z) + s_b[c]);
                    qv[c] = (int)fmax(fmin(v, 268435456.0), -268435456.0);
                }
                const int4 q = make_int4(qv[0], qv[1], qv[2], 0);
                if (it == 0) {
                    ch = true;
                } else {
                    const int4 o = qb[t];
                    ch |= o.x != q.x || o.y != q.y || o.z != q.z;
                }
                qb[t] = q;
            }
            if (ch) s_changed = 1;
            __syncthreads();
            if (!s_changed) break;
            long long acc = 0;
            for (int t = wave; t < ns; t += NW) {
                const int4 q = qb[t];
                const int nn = icp_nn(s, q, a.rq, a.rq2, label_mode ? s.labels : nullptr, a.label, a.box, lane);
                if (nn >= 0) {
                    const int4 c = gld(s.opt + nn);
                    if (lane < kIcpSums) acc += icp_term(lane, q, c);
                }
            }
            if (lane < kIcpSums) s_red[wave][lane] = acc;
            __syncthreads();
            if (tid < kIcpSums) {
                long long z = 0;
                for (int v = 0; v < NW; ++v) z += s_red[v][tid];
                s_red[0][tid] = z;
            }
            __syncthreads();
            if (tid == 0) {
                int stop = 0;
                matched = (int)s_red[0][0];
                if (s_red[0][0] < a.min_points) stop = 1;
                else if (icp_update(s_red[0], a.dof, u, s_A, s_b)) stop = 1;
                else iters = it + 1;
                s_stop = stop;
            }
            __syncthreads();
            if (s_stop) break;
        }
        if (tid == 0) {
            float *out = a.refined + 12 * (size_t)p;
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c)
                    out[4 * r + c] = (float)((s_A[3 * r] * (double)P[c] + s_A[3 * r + 1] * (double)P[4 + c])
                                             + s_A[3 * r + 2] * (double)P[8 + c]);
                const double t = ((s_A[3 * r] * (16.0 * (double)P[3]) + s_A[3 * r + 1] * (16.0 * (double)P[7]))
                                  + s_A[3 * r + 2] * (16.0 * (double)P[11])) + s_b[r];
                out[4 * r + 3] = (float)(t / 16.0);
            }
            if (a.iters) a.iters[p] = iters;
            if (a.matched) a.matched[p] = matched;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ pose proposals

// 6-DoF pose proposals (Sec. V-B "Pose Proposal Generation"): pose p is
// viewpoint i, in-plane angle k and depth t, p = (i N + k) T + t.  Viewpoint
// i of M on the Fibonacci lattice, z_i = 1 - (2 i + 1) / M at longitude
// i pi (3 - sqrt 5): the camera sits in direction v_i from the object, so
// the rotation takes v_i to the camera's -z axis (rows b1, b2, b3 with
// b3 = -v_i and b1 along z_obj x b3, or y_obj x b3 near the poles), then
// turns by 2 pi k / N about the optical axis.  The translation puts the
// object's centre (its mesh's AABB centre c) on the ray through the label
// box centre at depth z_t: t = z_t ray - R c.
__global__ void proposal_kernel(ProposalArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int t = p % a.T, k = (p / a.T) % a.N, i = p / (a.T * a.N);
    const double pi = 3.14159265358979323846;
    const double vz = 1.0 - (double)(2 * i + 1) / (double)a.M;
    const double r = sqrt(fmax(0.0, 1.0 - vz * vz));
    const double phi = (double)i * (pi * (3.0 - sqrt(5.0)));
    const double v[3] = {r * cos(phi), r * sin(phi), vz};
    const double b3[3] = {-v[0], -v[1], -v[2]};
    const double up[3] = {0.0, fabs(vz) > 0.999 ? 1.0 : 0.0, fabs(vz) > 0.999 ? 0.0 : 1.0};
    double b1[3] = {up[1] * b3[2] - up[2] * b3[1], up[2] * b3[0] - up[0] * b3[2], up[0] * b3[1] - up[1] * b3[0]};
    const double nb = sqrt((b1[0] * b1[0] + b1[1] * b1[1]) + b1[2] * b1[2]);
    for (int c = 0; c < 3; ++c) b1[c] = b1[c] / nb;
    const double b2[3] = {b3[1] * b1[2] - b3[2] * b1[1], b3[2] * b1[0] - b3[0] * b1[2], b3[0] * b1[1] - b3[1] * b1[0]};
    const double th = 2.0 * pi * (double)k / (double)a.N;
    const double co = cos(th), si = sin(th);
    const double z = a.zmin + (double)t * a.step;
    float *o = a.out + 12 * (size_t)p;
    for (int c = 0; c < 3; ++c) {
        o[c] = (float)(co * b1[c] - si * b2[c]);
        o[4 + c] = (float)(si * b1[c] + co * b2[c]);
        o[8 + c] = (float)b3[c];
    }
    const double ray[3] = {z * ((a.uc - (double)a.cx) / (double)a.fx), z * ((a.vc - (double)a.cy) / (double)a.fy), z};
    for (int r = 0; r < 3; ++r) {
        const double R0 = r == 0 ? co * b1[0] - si * b2[0] : (r == 1 ? si * b1[0] + co * b2[0] : b3[0]);
        const double R1 = r == 0 ? co * b1[1] - si * b2[1] : (r == 1 ? si * b1[1] + co * b2[1] : b3[1]);
        const double R2 = r == 0 ? co * b1[2] - si * b2[2] : (r == 1 ? si * b1[2] + co * b2[2] : b3[2]);
        o[4 * r + 3] = (float)(ray[r] - ((R0 * a.centre[0] + R1 * a.centre[1]) + R2 * a.centre[2]));
    }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_proposals(const ProposalArgs &a, hipStream_t st)
{
    if (a.n > 0) proposal_kernel<<<(a.n + 255) / 256, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_icp(const IcpArgs &a, int grid, hipStream_t st)
{
    icp_zero_kernel<<<1, 1, 0, st>>>(a.cursor);
    icp_kernel<1024><<<grid, 1024, (size_t)a.lds_words * 4, st>>>(a);
    return hipGetLastError();
}

hipError_t prepare_icp_kernel(int lds_per_group, int *lds_words)
{
    const void *f = (const void *)icp_kernel<1024>;
    hipFuncAttributes at{};
    hipError_t e = hipFuncGetAttributes(&at, f);
    if (e != hipSuccess) return e;
    const int dyn = lds_per_group - (int)at.sharedSizeBytes;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    *lds_words = e == hipSuccess ? dyn / 4 : 0;
    return e;
}

}  // namespace perch
