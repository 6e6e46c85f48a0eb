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
// GICP: 21 upper entries of the 6x6 Gauss-Newton matrix, then 6 of its
// right-hand side, in 64-bit fixed point (times 1024, rounded).
constexpr int kGicpSums = 27;
constexpr int kRedSums = 28;

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

// ------------------------------------------------------------------ GICP

// int4 arrays per work-group slot: source points, mapped points (with the
// match), and for GICP the source normals.
__host__ __device__ constexpr int gicp_slots(int method) { return method == 1 ? 3 : 2; }

// Integer normal direction of the point at pixel (i, j) of a depth image
// (depth(i', j') in mm, 0 = none): the cross product of the differences of
// the 1/16 mm points of the row and column neighbours, when all four exist
// inside the image, lie within `gap` mm of the pixel's depth and differ by
// at most 2^14 units per axis; 0 when there is none.
template <class Depth>
__device__ int pixel_normal(const SceneDev &s, int i, int j, int gap, Depth depth, int c[3])
{
    if (i < 1 || j < 1 || i > s.W - 2 || j > s.H - 2) return 0;
    const int d = depth(i, j);
    const int ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
    int p[4][3];
    for (int k = 0; k < 4; ++k) {
        const int dn = depth(ni[k], nj[k]);
        if (d == 0 || dn == 0 || dn - d > gap || d - dn > gap) return 0;
        p[k][0] = (int)rint(gld(s.kx + ni[k]) * (double)dn);
        p[k][1] = (int)rint(gld(s.ky + nj[k]) * (double)dn);
        p[k][2] = 16 * dn;
    }
    int ex[3], ey[3];
    for (int a = 0; a < 3; ++a) {
        ex[a] = p[1][a] - p[0][a];
        ey[a] = p[3][a] - p[2][a];
        if (ex[a] > 16384 || ex[a] < -16384 || ey[a] > 16384 || ey[a] < -16384) return 0;
    }
    c[0] = ex[1] * ey[2] - ex[2] * ey[1];
    c[1] = ex[2] * ey[0] - ex[0] * ey[2];
    c[2] = ex[0] * ey[1] - ex[1] * ey[0];
    return c[0] != 0 || c[1] != 0 || c[2] != 0;
}

__device__ __forceinline__ void unit_of(const int c[3], double n[3])
{
    const double x = (double)c[0], y = (double)c[1], z = (double)c[2];
    const double l = sqrt((x * x + y * y) + z * z);
    n[0] = x / l;
    n[1] = y / l;
    n[2] = z / l;
}

// Term j (of kGicpSums) of one match q -> c: with the plane covariances
// I - (1 - 1/1024) n n^T of the source normal turned by A and of the target
// normal (I without one), M = (C_a + C_b)^-1 by the adjugate, K = -[q - mu]x
// and e = c - q, the Gauss-Newton matrix [[K^T M K, K^T M], [M K, M]] (upper
// entries row by row) and right-hand side [K^T M e; M e], times 1024, rounded.
__device__ long long gicp_term(int j, int4 q, int4 c, const long long mu[3], int has_a, const double na[3],
                               int has_b, const double nb[3], const double *A)
{
    const double eps = 1.0 / 1024.0;
    double ra[3] = {0.0, 0.0, 0.0};
    if (has_a)
        for (int r = 0; r < 3; ++r) ra[r] = (A[3 * r] * na[0] + A[3 * r + 1] * na[1]) + A[3 * r + 2] * na[2];
    const double ka = has_a ? 1.0 - eps : 0.0, kb = has_b ? 1.0 - eps : 0.0;
    double S[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            const double sa = (r == k ? 1.0 : 0.0) - ka * (ra[r] * ra[k]);
            const double sb = (r == k ? 1.0 : 0.0) - kb * (nb[r] * nb[k]);
            S[r][k] = sa + sb;
        }
    double adj[3][3];
    adj[0][0] = S[1][1] * S[2][2] - S[1][2] * S[2][1];
    adj[0][1] = S[0][2] * S[2][1] - S[0][1] * S[2][2];
    adj[0][2] = S[0][1] * S[1][2] - S[0][2] * S[1][1];
    adj[1][0] = S[1][2] * S[2][0] - S[1][0] * S[2][2];
    adj[1][1] = S[0][0] * S[2][2] - S[0][2] * S[2][0];
    adj[1][2] = S[0][2] * S[1][0] - S[0][0] * S[1][2];
    adj[2][0] = S[1][0] * S[2][1] - S[1][1] * S[2][0];
    adj[2][1] = S[0][1] * S[2][0] - S[0][0] * S[2][1];
    adj[2][2] = S[0][0] * S[1][1] - S[0][1] * S[1][0];
    const double det = (S[0][0] * adj[0][0] + S[0][1] * adj[1][0]) + S[0][2] * adj[2][0];
    double M[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) M[r][k] = adj[r][k] / det;
    const double x = (double)((long long)q.x - mu[0]), y = (double)((long long)q.y - mu[1]),
                 z = (double)((long long)q.z - mu[2]);
    const double Kq[3][3] = {{0.0, z, -y}, {-z, 0.0, x}, {y, -x, 0.0}};
    const double e[3] = {(double)(c.x - q.x), (double)(c.y - q.y), (double)(c.z - q.z)};
    double MK[3][3], Me[3];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) MK[r][k] = (M[r][0] * Kq[0][k] + M[r][1] * Kq[1][k]) + M[r][2] * Kq[2][k];
        Me[r] = (M[r][0] * e[0] + M[r][1] * e[1]) + M[r][2] * e[2];
    }
    double v;
    if (j < 21) {
        // (r, k) of upper entry j, row by row
        int r = 0, k = j;
        while (k >= 6 - r) {
            k -= 6 - r;
            ++r;
        }
        k += r;
        if (r < 3 && k < 3) v = (Kq[0][r] * MK[0][k] + Kq[1][r] * MK[1][k]) + Kq[2][r] * MK[2][k];
        else if (r < 3) v = MK[k - 3][r];
        else v = M[r - 3][k - 3];
    } else if (j < 24) {
        const int r = j - 21;
        v = (Kq[0][r] * Me[0] + Kq[1][r] * Me[1]) + Kq[2][r] * Me[2];
    } else {
        v = Me[j - 24];
    }
    return (long long)rint(v * 1024.0);
}

// The GICP update from the fixed-point sums: H w = g by Cholesky (a pivot
// <= 0 returns 1, nothing changes), the rotation the unit quaternion
// (1, w/2) normalised, and (A, b) <- (Rc A, Rc (b - mu) + mu + t).
__device__ int gicp_update(const long long *z, const long long mu[3], double *A, double *b)
{
    double Hm[6][6], g[6];
    int t = 0;
    for (int r = 0; r < 6; ++r)
        for (int k = r; k < 6; ++k) {
            Hm[r][k] = (double)z[t++] / 1024.0;
            Hm[k][r] = Hm[r][k];
        }
    for (int r = 0; r < 6; ++r) g[r] = (double)z[t++] / 1024.0;
    double L[6][6];
    for (int r = 0; r < 6; ++r)
        for (int k = 0; k < 6; ++k) L[r][k] = 0.0;
    for (int jj = 0; jj < 6; ++jj) {
        double sjj = Hm[jj][jj];
        for (int k = 0; k < jj; ++k) sjj = sjj - L[jj][k] * L[jj][k];
        if (!(sjj > 0.0)) return 1;
        L[jj][jj] = sqrt(sjj);
        for (int i = jj + 1; i < 6; ++i) {
            double sij = Hm[i][jj];
            for (int k = 0; k < jj; ++k) sij = sij - L[i][k] * L[jj][k];
            L[i][jj] = sij / L[jj][jj];
        }
    }
    double yv[6], xv[6];
    for (int i = 0; i < 6; ++i) {
        double v = g[i];
        for (int k = 0; k < i; ++k) v = v - L[i][k] * yv[k];
        yv[i] = v / L[i][i];
    }
    for (int i = 5; i >= 0; --i) {
        double v = yv[i];
        for (int k = i + 1; k < 6; ++k) v = v - L[k][i] * xv[k];
        xv[i] = v / L[i][i];
    }
    const double h[3] = {xv[0] / 2.0, xv[1] / 2.0, xv[2] / 2.0};
    const double r = sqrt(1.0 + ((h[0] * h[0] + h[1] * h[1]) + h[2] * h[2]));
    const double qw = 1.0 / r, qx = h[0] / r, qy = h[1] / r, qz = h[2] / r;
    double R[3][3];
    R[0][0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    R[0][1] = 2.0 * (qx * qy - qz * qw);
    R[0][2] = 2.0 * (qx * qz + qy * qw);
    R[1][0] = 2.0 * (qx * qy + qz * qw);
    R[1][1] = 1.0 - 2.0 * (qx * qx + qz * qz);
    R[1][2] = 2.0 * (qy * qz - qx * qw);
    R[2][0] = 2.0 * (qx * qz - qy * qw);
    R[2][1] = 2.0 * (qy * qz + qx * qw);
    R[2][2] = 1.0 - 2.0 * (qx * qx + qy * qy);
    double An[9], bn[3];
    const double m[3] = {(double)mu[0], (double)mu[1], (double)mu[2]};
    const double e[3] = {b[0] - m[0], b[1] - m[1], b[2] - m[2]};
    for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c) An[3 * a + c] = (R[a][0] * A[c] + R[a][1] * A[3 + c]) + R[a][2] * A[6 + c];
        bn[a] = (((R[a][0] * e[0] + R[a][1] * e[1]) + R[a][2] * e[2]) + m[a]) + xv[3 + a];
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
    __shared__ long long s_red[NW][kRedSums];
    __shared__ double s_A[9], s_b[3];
    __shared__ long long s_mu[3];
    uint32_t *tile = a.tiles + (size_t)blockIdx.x * s.W * s.H;
    int4 *src = a.pts + (size_t)blockIdx.x * (gicp_slots(a.method)) * a.pts_cap;
    int4 *qb = src + a.pts_cap;
    int4 *nrm = qb + a.pts_cap;            // GICP: integer source normals (x, y, z, has)
    const bool gicp = a.method == 1;
    const int gap = a.rq >> 4;
    const bool mark = (s.flags & 2u) != 0;
    const bool label_mode = (s.flags & (3u << 4)) == (2u << 4);
    // Poses come through the cursor.  The loop is rotated by hand so that
    // its condition is a wave-uniform value (readfirstlane of the LDS copy)
    // and no branch on the thread index heads it; every exit from the
    // iteration loop below tests a readfirstlane value too.
    if (tid == 0) s_pose = atomicAdd(a.cursor, 1);
    __syncthreads();
    for (int p = __builtin_amdgcn_readfirstlane(s_pose); p < a.n;) {
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
            if (gicp) {
                // the render's own neighbours (any rendered pixel, on or off the stride grid)
                auto rdepth = [&](int ii, int jj) -> int {
                    if (ii < tx0 || jj < ty0 || ii >= tx0 + tw || jj >= ty0 + th) return 0;
                    const int kk = (jj - ty0) * tw + (ii - tx0);
                    const uint32_t kv = in_lds ? icp_lds[kk] : tld<true>(tile + kk);
                    return kv == kEmptyKey ? 0 : (int)(kv >> 16);
                };
                int c[3];
                const int has = pixel_normal(s, i, j, gap, rdepth, c);
                nrm[slot] = has ? make_int4(c[0], c[1], c[2], 1) : make_int4(0, 0, 0, 0);
            }
        }
        __syncthreads();
        const int ns = __builtin_amdgcn_readfirstlane(s_n);
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
            if (!__builtin_amdgcn_readfirstlane(s_changed)) break;
            long long acc = 0;
            for (int t = wave; t < ns; t += NW) {
                const int4 q = qb[t];
                const int nn = icp_nn(s, q, a.rq, a.rq2, label_mode ? s.labels : nullptr, a.label, a.box, lane);
                if (gicp && lane == 0) qb[t].w = nn;     // the match, for the second pass
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
                else if (gicp) {
                    // the centre of the matched points, rounded: exact integer sums
                    for (int c = 0; c < 3; ++c) s_mu[c] = (long long)rint((double)s_red[0][1 + c] / (double)s_red[0][0]);
                } else if (icp_update(s_red[0], a.dof, u, s_A, s_b)) {
                    stop = 1;
                } else {
                    iters = it + 1;
                }
                s_stop = stop;
            }
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(s_stop)) break;
            if (gicp) {
                // second pass: the Gauss-Newton terms of every match, one
                // wave per match, lane j summing term j
                const long long mu[3] = {s_mu[0], s_mu[1], s_mu[2]};
                long long gacc = 0;
                for (int t = wave; t < ns; t += NW) {
                    const int4 q = qb[t];
                    if (q.w < 0) continue;
                    const int4 c = gld(s.opt + q.w);
                    const int4 cs = nrm[t];
                    double na[3] = {0.0, 0.0, 0.0}, nb[3] = {0.0, 0.0, 0.0};
                    const int csv[3] = {cs.x, cs.y, cs.z};
                    if (cs.w) unit_of(csv, na);
                    const int pi = q.w % s.W, pj = q.w / s.W;
                    auto odepth = [&](int ii, int jj) -> int { return gld(s.depth + jj * s.W + ii); };
                    int cb[3];
                    const int has_b = pixel_normal(s, pi, pj, gap, odepth, cb);
                    if (has_b) unit_of(cb, nb);
                    if (lane < kGicpSums) gacc += gicp_term(lane, q, c, mu, cs.w, na, has_b, nb, s_A);
                }
                if (lane < kGicpSums) s_red[wave][lane] = gacc;
                __syncthreads();
                if (tid < kGicpSums) {
                    long long z = 0;
                    for (int v = 0; v < NW; ++v) z += s_red[v][tid];
                    s_red[0][tid] = z;
                }
                __syncthreads();
                if (tid == 0) {
                    const int stop = gicp_update(s_red[0], mu, s_A, s_b);
                    if (!stop) iters = it + 1;
                    s_stop = stop;
                }
                __syncthreads();
                if (__builtin_amdgcn_readfirstlane(s_stop)) break;
            }
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
            s_pose = atomicAdd(a.cursor, 1);
        }
        __syncthreads();
        p = __builtin_amdgcn_readfirstlane(s_pose);
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
