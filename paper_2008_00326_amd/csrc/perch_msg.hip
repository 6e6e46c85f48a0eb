// gfx950 kernels of the Monotone Scene Generation tree, the sequential search
// of the original PERCH that the variant 2.0-B of PERCH 2.0 keeps (Sec. III-B
// and its tree figure, Sec. VI-A).  A state's render lives in HBM as a few
// full-image planes; every successor of a state (one object in each of its
// candidate poses) is scored by one persistent launch:
//   1. rasterize the successor into a tile (LDS when it fits);
//   2. it is not monotone if it is nearer than the state's render on any
//      pixel both draw; its own points dR are its pixels the state leaves
//      empty, on the stride grid, less occluders (Eq. 3);
//   3. J_r of dR from the scene's nearest-neighbour table, with the colour
//      test of Eq. 4;
//   4. J_o over the observed points inside V(O) and outside every placed
//      object's volume: the nearest point of the composed render is the
//      nearer of the state's (kept per observed pixel with the state) and
//      the successor's own (searched in the tile), then Eq. 4.

#include "perch_device.h"

#include <math.h>

#include <algorithm>

namespace perch {

// ------------------------------------------------------------------ state images

__global__ __launch_bounds__(256) void msg_clear_kernel(SceneDev s, MsgState st)
{
    const int N = s.W * s.H;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
        st.depth[k] = 0;
        st.pts[k] = 0;
        if (st.rgb) st.rgb[k] = 0;
        st.cov[k] = 0;
        st.near[k] = ~0ULL;
    }
}

__global__ __launch_bounds__(256) void msg_keys_kernel(uint32_t *keys, int N)
{
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) keys[k] = kEmptyKey;
}

// One thread per triangle over the whole image.
__global__ __launch_bounds__(256) void msg_raster_kernel(MsgAddArgs a)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= a.m.nt) return;
    float P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = a.pose[k];
    raster_triangle<true>(a.s, a.m, P, t, 0, 0, a.s.W, a.s.H, a.keys);
}

// Append the rendered object to the state: pixels the state leaves empty
// take its depth and colour, and become points of R \ C on the stride grid
// unless the observed depth marks them as occluded (Eq. 3, the object's own
// label exempt); a pixel where it is nearer than the state flags the state
// as not monotone.  Observed points inside its volume become covered.
__global__ __launch_bounds__(256) void msg_compose_kernel(MsgAddArgs a)
{
    const SceneDev &s = a.s;
    const int N = s.W * s.H;
    const bool mark = (s.flags & 2u) != 0;
    const bool label_mode = (s.flags & (3u << 4)) == (2u << 4);
    const bool cyl = (s.flags & (3u << 4)) == (1u << 4);
    const double dl = (double)s.delta;
    float P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = a.pose[k];
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
        const int j = k / s.W, i = k - j * s.W;
        const uint32_t key = a.keys[k];
        if (key != kEmptyKey) {
            const int d = (int)(key >> 16);
            const int sd = a.st.depth[k];
            if (sd > 0) {
                if (d < sd) atomicOr(a.flag, 1);
            } else {
                a.st.depth[k] = (uint16_t)d;
                if (a.st.rgb) a.st.rgb[k] = triangle_colour(s, a.m, P, (int)(key & 0xFFFFu), i, j);
                bool pt = i % s.stride == 0 && j % s.stride == 0;
                if (pt && mark) {
                    const int dob = s.depth[k];
                    if (dob > 0 && 16 * dob + s.dq < 16 * d && (!(label_mode && s.labels) || s.labels[k] != a.label))
                        pt = false;
                }
                a.st.pts[k] = pt ? (uint16_t)d : (uint16_t)0;
            }
        }
        const int4 o = s.opt[k];
        if (o.z != kNoPoint && !a.st.cov[k]) {
            const bool in = label_mode ? (s.labels && s.labels[k] == a.label)
                                       : in_volume(a.m, P, o.x, o.y, o.z >> 4, dl, cyl);
            if (in) a.st.cov[k] = 1;
        }
    }
}

// Per observed pixel, the nearest point of the state's R \ C within delta:
// min (squared distance << 32 | pixel), ~0 when none.
__global__ __launch_bounds__(256) void msg_near_kernel(SceneDev s, MsgState st)
{
    const int N = s.W * s.H;
    const float dlw = s.delta + 0.25f;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < N; k += gridDim.x * 256) {
        const int4 o = s.opt[k];
        unsigned long long best = ~0ULL;
        if (o.z != kNoPoint) {
            const int j = k / s.W, i = k - j * s.W;
            const float iz = window_inv(o.z >> 4, dlw);
            const int wu = window_half(s.ax[i], iz, s.W), wv = window_half(s.ay[j], iz, s.H);
            const int i0 = max(i - wu, 0), i1 = min(i + wu, s.W - 1);
            const int j0 = max(j - wv, 0), j1 = min(j + wv, s.H - 1);
            for (int jj = j0; jj <= j1; ++jj)
                for (int ii = i0; ii <= i1; ++ii) {
                    const int u = jj * s.W + ii;
                    const int d = st.pts[u];
                    if (d == 0) continue;
                    const long long dx = (long long)rint(s.kx[ii] * (double)d) - o.x;
                    const long long dy = (long long)rint(s.ky[jj] * (double)d) - o.y;
                    const long long dz = 16LL * d - o.z;
                    const long long d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 <= (long long)s.dq2) {
                        const unsigned long long c = ((unsigned long long)d2 << 32) | (uint32_t)u;
                        best = c < best ? c : best;
                    }
                }
        }
        st.near[k] = best;
    }
}

// ------------------------------------------------------------------ successors

__global__ void msg_zero_kernel(int *cursor)
{
    if (threadIdx.x == 0) cursor[0] = 0;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void msg_kernel(MsgArgs a)
{
    const int tid = threadIdx.x;
    const SceneDev &s = a.s;
    const MeshDev &m = a.m;
    extern __shared__ uint32_t msg_lds[];
    __shared__ int s_pose, s_box[4], s_reg[4], s_bad, s_cnt[4];
    uint32_t *gtile = a.tiles + (size_t)blockIdx.x * s.W * s.H;
    const bool rgb = (s.flags & 1u) != 0;
    const bool mark = (s.flags & 2u) != 0;
    const bool label_mode = (s.flags & (3u << 4)) == (2u << 4);
    const bool cyl = (s.flags & (3u << 4)) == (1u << 4);
    const double dl = (double)s.delta;
    const float dlw = s.delta + 0.25f;
    // Poses come through the cursor; the loop is rotated by hand so that its
    // condition is a wave-uniform value and no branch on the thread index
    // heads it: with a divergent `if (tid == 0)` fetch at the top, the
    // compiler may send thread 0 alone round an outer loop to fetch the next
    // pose while the other lanes wait for it at the barrier, which they then
    // pass without it.
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
            } else if (!(zmax < 99.999)) {
                w = s.W;
                h = s.H;
            }
            s_box[0] = x0;
            s_box[1] = y0;
            s_box[2] = w;
            s_box[3] = h;
            // every observed pixel that may lie in V(O): the label's box, or
            // the projection of the grown box when it lies wholly in front of
            // the camera, else the whole image
            if (label_mode) {
                for (int c = 0; c < 4; ++c) s_reg[c] = a.vbox[c];
            } else {
                project_box(P, m.lo, m.hi, dl, s, &umin, &umax, &vmin, &vmax, &zmin, &zmax);
                if (zmin > 0.0) {
                    clip_box(umin, umax, vmin, vmax, s.W, s.H, &x0, &y0, &w, &h);
                } else {
                    x0 = y0 = 0;
                    w = s.W;
                    h = s.H;
                }
                s_reg[0] = x0;
                s_reg[1] = y0;
                s_reg[2] = w;
                s_reg[3] = h;
            }
            s_bad = 0;
            for (int c = 0; c < 4; ++c) s_cnt[c] = 0;
        }
        __syncthreads();
        const int tx0 = s_box[0], ty0 = s_box[1], tw = s_box[2], th = s_box[3];
        const int tpx = tw * th;
        const bool in_lds = tpx <= a.lds_words;
        const int tile_q = (tpx + 3) & ~3;
        const int4 *vcache = nullptr;
        if (in_lds) {
            for (int k = tid; k < tpx; k += BLOCK) msg_lds[k] = kEmptyKey;
            if (tpx > 0 && 4 * m.nv <= a.lds_words - tile_q) {
                int4 *vc = reinterpret_cast<int4 *>(msg_lds + tile_q);
                for (int v = tid; v < m.nv; v += BLOCK) vc[v] = pack_vtx(project_vertex(P, gld(m.verts + v), s));
                vcache = vc;
            }
        } else {
            for (int k = tid; k < tpx; k += BLOCK) tst<true>(gtile + k, kEmptyKey);
        }
        __syncthreads();
        if (tpx > 0)
            for (int t0 = 0; t0 < m.nt; t0 += BLOCK)
                if (t0 + tid < m.nt) {
                    if (in_lds) raster_triangle<false>(s, m, P, t0 + tid, tx0, ty0, tw, th, msg_lds, vcache);
                    else raster_triangle<true>(s, m, P, t0 + tid, tx0, ty0, tw, th, gtile);
                }
        __syncthreads();
        // monotonicity, dR \ C (the tile keeps only its pixels) and J_r
        int bad = 0, cr = 0, cn = 0;
        for (int k = tid; k < tpx; k += BLOCK) {
            const uint32_t key = in_lds ? msg_lds[k] : tld<true>(gtile + k);
            if (key == kEmptyKey) continue;
            const int ty = k / tw, tx = k - ty * tw;
            const int i = tx0 + tx, j = ty0 + ty, d = (int)(key >> 16);
            const int pix = j * s.W + i;
            const int sd = gld(a.st.depth + pix);
            bool keep = true;
            if (sd > 0) {
                bad |= d < sd;
                keep = false;
            } else if (i % s.stride != 0 || j % s.stride != 0) {
                keep = false;
            } else if (mark) {
                const int dob = gld(s.depth + pix);
                if (dob > 0 && 16 * dob + s.dq < 16 * d && (!(label_mode && s.labels) || s.labels[pix] != a.label))
                    keep = false;
            }
            if (!keep) {
                if (in_lds) msg_lds[k] = kEmptyKey;
                else tst<true>(gtile + k, kEmptyKey);
                continue;
            }
            ++cn;
            int nn;
            if (s.flags & kHashFlag) {
                nn = hash_nn(s, (int)rint(gld(s.kx + i) * (double)d), (int)rint(gld(s.ky + j) * (double)d), 16 * d);
            } else {
                const int2 tr = gld(s.thdr + pix);
                const int e = d - (tr.y & 0xFFFF);
                nn = (e >= 0 && e < (int)((uint32_t)tr.y >> 16)) ? gld(s.tnn + tr.x + e) : -1;
            }
            bool out = nn < 0;
            if (!out && rgb)
                out = ciede2000(srgb_to_lab(triangle_colour(s, m, P, (int)(key & 0xFFFFu), i, j)), gld(s.olab + nn)) > s.tau;
            cr += out;
        }
        if (bad) s_bad = 1;
        if (cr) atomicAdd(&s_cnt[0], cr);
        if (cn) atomicAdd(&s_cnt[2], cn);
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(s_bad)) {
            // J_o over the observed points of V(O) outside every placed volume
            const int rx0 = s_reg[0], ry0 = s_reg[1], rw = s_reg[2], rh = s_reg[3];
            const int rpx = rw * rh;
            int co = 0, cq = 0;
            for (int q = tid; q < rpx; q += BLOCK) {
                const int ry = q / rw, rx = q - ry * rw;
                const int i = rx0 + rx, j = ry0 + ry, pix = j * s.W + i;
                const int4 o = gld(s.opt + pix);
                if (o.z == kNoPoint || gld(a.st.cov + pix)) continue;
                const bool in = label_mode ? (s.labels && gld(s.labels + pix) == a.label)
                                           : in_volume(m, P, o.x, o.y, o.z >> 4, dl, cyl);
                if (!in) continue;
                ++cq;
                unsigned long long best = gld(a.st.near + pix);
                if (tpx > 0) {
                    const float iz = window_inv(o.z >> 4, dlw);
                    const int wu = window_half(gld(s.ax + i), iz, s.W), wv = window_half(gld(s.ay + j), iz, s.H);
                    const int i0 = max(i - wu, tx0), i1 = min(i + wu, tx0 + tw - 1);
                    const int j0 = max(j - wv, ty0), j1 = min(j + wv, ty0 + th - 1);
                    for (int jj = j0; jj <= j1; ++jj)
                        for (int ii = i0; ii <= i1; ++ii) {
                            const int kk = (jj - ty0) * tw + (ii - tx0);
                            const uint32_t key = in_lds ? msg_lds[kk] : tld<true>(gtile + kk);
                            if (key == kEmptyKey) continue;
                            const int d = (int)(key >> 16);
                            const long long dx = (long long)rint(gld(s.kx + ii) * (double)d) - o.x;
                            const long long dy = (long long)rint(gld(s.ky + jj) * (double)d) - o.y;
                            const long long dz = 16LL * d - o.z;
                            const long long d2 = dx * dx + dy * dy + dz * dz;
                            if (d2 <= (long long)s.dq2) {
                                const unsigned long long c = ((unsigned long long)d2 << 32) | (uint32_t)(jj * s.W + ii);
                                best = c < best ? c : best;
                            }
                        }
                }
                bool out = best == ~0ULL;
                if (!out && rgb) {
                    // the nearest point is the state's or the successor's own
                    const int u = (int)(best & 0xFFFFFFFFu);
                    uint32_t c;
                    if (gld(a.st.pts + u) > 0) {
                        c = gld(a.st.rgb + u);
                    } else {
                        const int uj = u / s.W, ui = u - uj * s.W;
                        const int kk = (uj - ty0) * tw + (ui - tx0);
                        const uint32_t key = in_lds ? msg_lds[kk] : tld<true>(gtile + kk);
                        c = triangle_colour(s, m, P, (int)(key & 0xFFFFu), ui, uj);
                    }
                    out = ciede2000(gld(s.olab + pix), srgb_to_lab(c)) > s.tau;
                }
                co += out;
            }
            if (co) atomicAdd(&s_cnt[1], co);
            if (cq) atomicAdd(&s_cnt[3], cq);
        }
        __syncthreads();
        if (tid == 0) {
            const bool ok = !s_bad;
            a.valid[p] = ok;
            a.jr[p] = ok ? s_cnt[0] : 0;
            a.jo[p] = ok ? s_cnt[1] : 0;
            if (a.nr) a.nr[p] = ok ? s_cnt[2] : 0;
            if (a.nq) a.nq[p] = ok ? s_cnt[3] : 0;
            s_pose = atomicAdd(a.cursor, 1);
        }
        __syncthreads();
        p = __builtin_amdgcn_readfirstlane(s_pose);
    }
}

// ------------------------------------------------------------------ launches

hipError_t upload_msg_colour_table(const float *lin256)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lin), lin256, 256 * sizeof(float));
}

static int pixel_grid(int N)
{
    return std::max(1, std::min((N + 255) / 256, 4096));
}

hipError_t msg_state_clear(const SceneDev &s, const MsgState &st, hipStream_t stream)
{
    msg_clear_kernel<<<pixel_grid(s.W * s.H), 256, 0, stream>>>(s, st);
    return hipGetLastError();
}

hipError_t msg_state_add(const MsgAddArgs &a, hipStream_t stream)
{
    const int N = a.s.W * a.s.H;
    msg_keys_kernel<<<pixel_grid(N), 256, 0, stream>>>(a.keys, N);
    if (a.m.nt > 0) msg_raster_kernel<<<(a.m.nt + 255) / 256, 256, 0, stream>>>(a);
    msg_compose_kernel<<<pixel_grid(N), 256, 0, stream>>>(a);
    return hipGetLastError();
}

hipError_t msg_state_near(const SceneDev &s, const MsgState &st, hipStream_t stream)
{
    msg_near_kernel<<<pixel_grid(s.W * s.H), 256, 0, stream>>>(s, st);
    return hipGetLastError();
}

hipError_t launch_msg(const MsgArgs &a, int grid, hipStream_t stream)
{
    msg_zero_kernel<<<1, 1, 0, stream>>>(a.cursor);
    msg_kernel<512><<<grid, 512, (size_t)a.lds_words * 4, stream>>>(a);
    return hipGetLastError();
}

hipError_t prepare_msg_kernel(int lds_per_group, int *lds_words)
{
    const void *f = (const void *)msg_kernel<512>;
    hipFuncAttributes at{};
    hipError_t e = hipFuncGetAttributes(&at, f);
    if (e != hipSuccess) return e;
    const int dyn = lds_per_group - (int)at.sharedSizeBytes;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    *lds_words = e == hipSuccess ? dyn / 4 : 0;
    return e;
}

}  // namespace perch
