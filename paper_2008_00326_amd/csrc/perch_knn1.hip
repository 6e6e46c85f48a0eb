// kNN I (Sec. IV-A "Parallel Cost Computation"): the paper's fully parallel
// neighbour search, which computes every distance between a pose's rendered
// points and the input cloud into one two-dimensional array, then reduces
// it.  Kept as a comparison baseline beside the scene's neighbour table: it
// gives the same neighbours (exact integer distances, ties to the lower
// pixel index), so the same costs, at the memory the paper names as its
// limit -- L x I x 4 bytes per pose.  One pose at a time:
//   1. rasterize over the image and compact R \ C (stride grid, occluders);
//   2. D[r][i] = squared distance of rendered point r to observed point i;
//   3. per row, the nearest observed point within delta: J_r (Eq. 2, Eq. 4),
//      and with nearest-neighbour J_o marking, the mark of that point;
//   4. per column (observed points inside V), the nearest rendered point
//      within delta, read down the column: J_o (Eq. 3, Eq. 4).

#include "perch_device.h"

#include <math.h>

namespace perch {

// Observed points: the pixels with a reading, in any order (keys carry the
// pixel index, so ties resolve by pixel whatever the order).
__global__ __launch_bounds__(256) void knn1_obs_kernel(SceneDev s, int *obs, int *n_obs)
{
    const int N = s.W * s.H;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256)
        if (s.opt[k].z != kNoPoint) obs[atomicAdd(n_obs, 1)] = k;
}

__global__ __launch_bounds__(256) void knn1_clear_kernel(uint32_t *keys, int N, int *counts)
{
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) keys[k] = kEmptyKey;
    if (blockIdx.x == 0 && threadIdx.x < 4) counts[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void knn1_raster_kernel(Knn1Args a, int p)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= a.m.nt) return;
    float P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = a.poses[12 * (size_t)p + k];
    raster_triangle<true>(a.s, a.m, P, t, 0, 0, a.s.W, a.s.H, a.keys);
}

// R \ C as a list of points (X, Y, Z in 1/16 mm, pixel); colours by pixel.
__global__ __launch_bounds__(256) void knn1_points_kernel(Knn1Args a, int p)
{
    const SceneDev &s = a.s;
    const int N = s.W * s.H;
    const bool mark = (s.flags & 2u) != 0;
    const bool label_mode = (s.flags & (3u << 4)) == (2u << 4);
    const bool rgb = (s.flags & 1u) != 0;
    float P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = a.poses[12 * (size_t)p + k];
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
        const uint32_t key = a.keys[k];
        if (key == kEmptyKey) continue;
        const int j = k / s.W, i = k - j * s.W, d = (int)(key >> 16);
        if (i % s.stride != 0 || j % s.stride != 0) continue;
        if (mark) {
            const int dob = s.depth[k];
            if (dob > 0 && 16 * dob + s.dq < 16 * d && (!(label_mode && s.labels) || s.labels[k] != a.label))
                continue;
        }
        const int slot = atomicAdd(&a.counts[0], 1);
        a.pts[slot] = make_int4((int)rint(s.kx[i] * (double)d), (int)rint(s.ky[j] * (double)d), 16 * d, k);
        if (rgb) a.pcol[k] = triangle_colour(s, a.m, P, (int)(key & 0xFFFFu), i, j);
    }
}

// The two-dimensional array of kNN I: every (rendered, observed) pair's
// squared distance, saturated to 32 bits (only those within delta matter).
__global__ __launch_bounds__(256) void knn1_dist_kernel(Knn1Args a, int L)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n_obs) return;
    const int4 o = a.s.opt[a.obs[i]];
    for (int r = blockIdx.y; r < L; r += gridDim.y) {
        const int4 q = a.pts[r];
        const long long dx = (long long)q.x - o.x, dy = (long long)q.y - o.y, dz = (long long)q.z - o.z;
        const long long d2 = dx * dx + dy * dy + dz * dz;
        a.dist[(size_t)r * a.n_obs + i] = d2 > 0xFFFFFFFFLL ? 0xFFFFFFFFu : (uint32_t)d2;
    }
}

__device__ __forceinline__ unsigned long long wave_min64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long w = __shfl_xor(v, off, 64);
        v = w < v ? w : v;
    }
    return v;
}

// One wave per row: the rendered point's nearest observed point within delta.
__global__ __launch_bounds__(256) void knn1_rows_kernel(Knn1Args a, int L)
{
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= L) return;
    const uint32_t *row = a.dist + (size_t)r * a.n_obs;
    unsigned long long best = ~0ULL;
    for (int i = lane; i < a.n_obs; i += 64) {
        const uint32_t d2 = row[i];
        if (d2 <= (uint32_t)a.s.dq2) {
            const unsigned long long c = ((unsigned long long)d2 << 32) | (uint32_t)a.obs[i];
            best = c < best ? c : best;
        }
    }
    best = wave_min64(best);
    if (lane != 0) return;
    const bool rgb = (a.s.flags & 1u) != 0;
    const bool nnm = (a.s.flags & (1u << 6)) != 0;
    bool out = best == ~0ULL;
    const int nn = out ? -1 : (int)(best & 0xFFFFFFFFu);
    if (!out && rgb) out = ciede2000(srgb_to_lab(a.pcol[a.pts[r].w]), a.s.olab[nn]) > a.s.tau;
    if (out) atomicAdd(&a.counts[1], 1);
    else if (nnm) a.marked[nn] = 1;
}

// One thread per observed point: inside V(O), then (exact J_o) the nearest
// rendered point within delta down its column, or (nearest-neighbour
// marking) its mark.
__global__ __launch_bounds__(256) void knn1_cols_kernel(Knn1Args a, int p, int L)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n_obs) return;
    const SceneDev &s = a.s;
    const int pix = a.obs[i];
    const int4 o = s.opt[pix];
    const bool label_mode = (s.flags & (3u << 4)) == (2u << 4);
    const bool cyl = (s.flags & (3u << 4)) == (1u << 4);
    float P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = a.poses[12 * (size_t)p + k];
    const bool in = label_mode ? (s.labels && s.labels[pix] == a.label)
                               : in_volume(a.m, P, o.x, o.y, o.z >> 4, (double)s.delta, cyl);
    if (!in) return;
    atomicAdd(&a.counts[3], 1);
    bool out;
    if (s.flags & (1u << 6)) {
        out = !a.marked[pix];
    } else {
        unsigned long long best = ~0ULL;
        for (int r = 0; r < L; ++r) {
            const uint32_t d2 = a.dist[(size_t)r * a.n_obs + i];
            if (d2 <= (uint32_t)s.dq2) {
                const unsigned long long c = ((unsigned long long)d2 << 32) | (uint32_t)a.pts[r].w;
                best = c < best ? c : best;
            }
        }
        out = best == ~0ULL;
        if (!out && (s.flags & 1u))
            out = ciede2000(s.olab[pix], srgb_to_lab(a.pcol[(int)(best & 0xFFFFFFFFu)])) > s.tau;
    }
    if (out) atomicAdd(&a.counts[2], 1);
}

__global__ void knn1_write_kernel(Knn1Args a, int p)
{
    if (threadIdx.x != 0) return;
    a.jr[p] = a.counts[1];
    a.jo[p] = a.counts[2];
    if (a.nr) a.nr[p] = a.counts[0];
    if (a.nq) a.nq[p] = a.counts[3];
}

__global__ __launch_bounds__(256) void knn1_unmark_kernel(uint8_t *marked, int N)
{
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) marked[k] = 0;
}

// ------------------------------------------------------------------ launches

static int grid_of(int n)
{
    return n <= 0 ? 1 : (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
}

hipError_t upload_knn1_colour_table(const float *lin256)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lin), lin256, 256 * sizeof(float));
}

hipError_t knn1_observed(const SceneDev &s, int *obs, int *n_obs, hipStream_t st)
{
    knn1_obs_kernel<<<grid_of(s.W * s.H), 256, 0, st>>>(s, obs, n_obs);
    return hipGetLastError();
}

hipError_t knn1_render(const Knn1Args &a, int p, hipStream_t st)
{
    const int N = a.s.W * a.s.H;
    knn1_clear_kernel<<<grid_of(N), 256, 0, st>>>(a.keys, N, a.counts);
    if (a.marked) knn1_unmark_kernel<<<grid_of(N), 256, 0, st>>>(a.marked, N);
    if (a.m.nt > 0) knn1_raster_kernel<<<(a.m.nt + 255) / 256, 256, 0, st>>>(a, p);
    knn1_points_kernel<<<grid_of(N), 256, 0, st>>>(a, p);
    return hipGetLastError();
}

hipError_t knn1_score(const Knn1Args &a, int p, int L, hipStream_t st)
{
    if (L > 0 && a.n_obs > 0) {
        knn1_dist_kernel<<<dim3((a.n_obs + 255) / 256, L < 32768 ? L : 32768), 256, 0, st>>>(a, L);
        knn1_rows_kernel<<<(L + 3) / 4, 256, 0, st>>>(a, L);
    }
    if (a.n_obs > 0) knn1_cols_kernel<<<(a.n_obs + 255) / 256, 256, 0, st>>>(a, p, L);
    knn1_write_kernel<<<1, 64, 0, st>>>(a, p);
    return hipGetLastError();
}

}  // namespace perch
