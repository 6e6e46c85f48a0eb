/*
 * PERCH 2.0 pose-scoring oracle: a plain, slow, obviously-correct CPU model.
 *
 * TEST INFRASTRUCTURE ONLY.  The library built from this file may be loaded
 * by the test-suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark, nowhere else.  It shares no code, header, table or constant
 * generator with the HIP path, and it does not include any of the HIP path's
 * headers.
 *
 * What it computes, following Agarwal, Han, Likhachev, "PERCH 2.0: Fast and
 * Accurate GPU-based Perception via Search for Object Pose Estimation":
 *   - Sec. III-B, Eq. 1: J = J_o + J_r, an unweighted sum of outlier counts.
 *   - Sec. III-B, Eq. 2: a point is an outlier w.r.t. a cloud iff its nearest
 *     point in that cloud is farther than delta (the sensor resolution).
 *   - Sec. IV-A "Parallel Search", Eq. 3: J_r counts rendered points that are
 *     not occluders; J_o counts observed points inside the object's volume
 *     V(O); the occluders C are found from the input depth image.
 *   - Sec. IV-B, Eq. 4: in RGB mode a point that does have a neighbour within
 *     delta is still an outlier when the CIEDE2000 difference between its
 *     CIELAB colour and its match's exceeds tau_c; applied to rendered and
 *     observed points alike ("or vice-versa").
 *   - Sec. IV-A "Parallel Rendering": every candidate pose is rendered into
 *     depth (and colour) and back-projected to a point cloud, downsampled in
 *     image space.
 *   - Sec. IV-A "Parallel Search": the per-object minimum-cost pose.
 *   - Sec. V-C: with segmentation labels, J_o counts the observed points that
 *     carry the object's label, and only pixels of another label occlude.
 *
 * The paper fixes no rasterization, quantization or precision convention.
 * The readings followed here (the HIP path follows the same ones):
 *   R1 Transform: Xc = ((R00 x + R01 y) + R02 z) + t0 in binary64 from binary32
 *      inputs, left to right, no fused multiply-add.
 *   R2 Projection: iz = 1/Zc; u = ((fx Xc) iz) + cx; U = rint(256 u) (8
 *      sub-pixel bits).  Integer pixel coordinates are pixel centres.  A
 *      triangle is dropped if any vertex has Zc < 100 mm or |256 u| > 2^24.
 *   R3 Edge functions E_ab(p) = (b.y-a.y)(p.x-a.x) - (b.x-a.x)(p.y-a.y) in
 *      int64; area A = E_01(v2); a triangle is drawn iff A > 0 (the mesh is
 *      counter-clockwise about the outward normal and the screen y axis points
 *      down).  A pixel is covered iff each edge has E > 0, or E == 0 and the
 *      edge is top-left (dy > 0, or dy == 0 and dx < 0).
 *   R4 Depth: t_k = w_k * iz_k, s = (t0 + t1) + t2, z = A / s, d = rint(z) in
 *      millimetres; the fragment is kept iff 1 <= d <= 65534.  Visibility
 *      uses a 16-bit millimetre depth buffer with triangles drawn in index
 *      order under a strict less-than test: the fragment with the smallest
 *      (d, triangle index) wins.
 *   R5 Colour: c = ((t0 c0 + t1 c1) + t2 c2) / s per channel, rint, clamped
 *      to [0, 255].
 *   R6 Occluders: a rendered pixel is dropped iff the observed depth d_o > 0
 *      and 16 d_o + dq < 16 d (dq = rint(16 delta)); in label mode only an
 *      observed pixel whose label differs from the object's label occludes.
 *   R7 Points in 1/16 mm: kx[i] = ((i - cx) 16) / fx, Xq = rint(kx[i] d),
 *      likewise Yq with ky[j], Zq = 16 d.  R keeps pixels with i and j
 *      multiples of the stride.
 *   R8 Neighbours: dx^2 + dy^2 + dz^2 <= dq^2 in exact integers.
 *   R9 In RGB mode the match is the nearest neighbour, ties broken by the
 *      lower row-major pixel index.  The colour decision dE00(point, match)
 *      > tau_c is taken in binary32, the precision of the GPU path; the
 *      binary64 colour functions exist to pin the binary32 ones.
 *   R10 Volume: the object-frame AABB of the mesh, inflated by delta, tested
 *      in binary64 on q = R^T (P - t) with P = (Xq, Yq, Zq) / 16.  The
 *      inscribed-cylinder volume (Table I's conservative V) takes the
 *      cylinder whose axis is the object z axis through the AABB's centre in
 *      x and y, with radius the smaller half-extent in x and y and the AABB's
 *      z range; it is inflated by delta like the box: (q0 - c0)^2 +
 *      (q1 - c1)^2 <= (rho + delta)^2 and lo2 - delta <= q2 <= hi2 + delta.
 *   R12 Nearest-neighbour marking of J_o (the paper's own J_o kernel, Sec.
 *      IV-A "Parallel Cost Computation"): optionally an observed point inside
 *      V is explained iff it is the nearest observed point (R9) within delta
 *      of some point of R minus C that passes its own colour test; otherwise
 *      it is an outlier.  No further colour test applies to it.
 *   R11 Selection: lowest J; ties go to the lowest pose index.
 *
 * ICP refinement (Sec. IV-A "Parallel M2M GICP" and Sec. VI-A: each pose is
 * aligned to the observed cloud by ICP, then rendered and scored again; the
 * 3-DoF experiments use point-to-point ICP).  The paper gives no
 * correspondence rule, update or stopping rule; this oracle reads them as:
 *   I1 Source: R minus C of the pose (R6, R7) on the ICP stride grid; target:
 *      every valid observed point or, with label volumes (Sec. V-C: the 6-DoF
 *      pipeline segments each object first), those carrying the object's
 *      label.  Integer 1/16 mm points.
 *   I2 Iteration k holds a camera-frame transform (A, b), b in 1/16 mm,
 *      starting at the identity.  Source point s maps to q with
 *      q_a = rint(((A_a0 sx + A_a1 sy) + A_a2 sz) + b_a).
 *   I3 The match c of q is its nearest observed point within rho: with
 *      rq = rint(16 rho), dx^2 + dy^2 + dz^2 <= rq^2 in exact integers, ties to
 *      the lower pixel index.  Unmatched points take no part.
 *   I4 Exact int64 sums over the matches: n, Sq, Sc, Sqq, Sqc.  Then, in
 *      binary64 in this order: mq = Sq / n, mc = Sc / n,
 *      S_ab = Sqq_ab - (Sq_a Sq_b) / n, H_ab = Sqc_ab - (Sq_a Sc_b) / n,
 *      w = (H12 - H21, H20 - H02, H01 - H10).
 *   I5 Update, a rotation Rc about mq and the image m' of mq:
 *      3-DoF (rotation about the pose's object z axis u, translation normal to
 *      u): the exact planar Procrustes solution, A' = (H00 + H11) + H22 - u.Hu,
 *      B = u.w, h = sqrt(A'^2 + B^2), (cos, sin) = (A'/h, B/h) (no rotation
 *      when h = 0), Rc = cos I + sin [u]x + (1 - cos) u u^T,
 *      m' = mq + (d - (u.d) u) with d = mc - mq.
 *      6-DoF: one Gauss-Newton step of the linearised rotation about mq,
 *      M w' = w with M = tr(S) I - S, solved by the adjugate (stop when
 *      det M <= 0), Rc from the unit quaternion (1, w'/2) / sqrt(1 + |w'/2|^2),
 *      m' = mc.
 *   I6 (A, b) <- (Rc A, Rc (b - mq) + m').
 *   I7 Before each iteration k > 0 ICP stops when the quantised q equal
 *      those of the previous iteration (the update would repeat); it stops
 *      after K iterations, and when fewer than min_points points match.
 *   I8 Refined pose: R' = A R_P, t' = (A (16 t_P) + b) / 16, rounded to
 *      binary32.
 * Products and sums are written left to right as above; no fused
 * multiply-add (as R1).
 *
 * GICP (Sec. IV-A "Parallel M2M GICP": each point's surface as a Gaussian),
 * 6-DoF, read as plane-to-plane GICP on image-structured clouds:
 *   G1 Normal of the point at pixel (i, j) of a depth image (the render for
 *      source points, the observed image for targets): with all four
 *      neighbours (i +- 1, j), (i, j +- 1) inside the image, with a reading,
 *      and within g = floor(rq / 16) mm of the pixel's depth, c = ex x ey
 *      where ex, ey are the differences of the neighbours' 1/16 mm points
 *      (R7) along the row and the column (exact integers; none when any
 *      component of ex or ey exceeds 2^14 or c = 0); n = c / |c|.
 *   G2 Covariance I - (1 - e) n n^T with e = 1/1024 (unit variance in the
 *      surface, e across it); I without a normal.
 *   G3 Matches as I2-I3 (mapped points rounded to 1/16 mm).
 *   G4 Centre mu = rint(sum q / n) per axis (exact integer sums).  Per match:
 *      q~ = q - mu, e = c - q, the source normal turned by the current
 *      rotation A, S = C_a + C_b, M = adj(S) / det(S), K = -[q~]x, and the
 *      Gauss-Newton terms of the increment (w, t) with q' = q + w x q~ + t:
 *      H = [[K^T M K, K^T M], [M K, M]], g = [K^T M e; M e].  The 21 upper
 *      entries of H and the 6 of g, each times 1024 and rounded, are summed
 *      exactly in 64 bits.
 *   G5 H w = g by Cholesky (pivots in order; a pivot <= 0 stops GICP), the
 *      rotation the unit quaternion (1, w/2) / sqrt(1 + |w/2|^2), and
 *      (A, b) <- (Rc A, Rc (b - mu) + mu + t).
 *   G6 Stops as I7 (no mapped point moved, fewer than min_points matches,
 *      K updates) and on a failed pivot; refined pose as I8.
 *
 * Monotone Scene Generation tree (the sequential search of the original
 * PERCH that the variant 2.0-B keeps, Sec. III-B and its tree figure, Sec.
 * VI-A), read as:
 *   M1 A state is a sequence of placed objects (object, candidate pose), each
 *      object at most once.  The root is empty; a successor appends one
 *      object not yet placed, in one of its candidate poses; states with
 *      every object placed are goals.
 *   M2 A state's render is its objects' renders (R4) composed in order: a
 *      pixel keeps the first object that draws it.  A successor is monotone
 *      iff the new object occludes none already placed: no pixel that both
 *      draw with the new depth strictly smaller.  Only monotone successors
 *      enter the tree.
 *   M3 The edge cost of appending object O at pose P to state S is J_r over
 *      O's own points dR (its pixels that no object of S draws, on the
 *      stride grid, less occluders by R6 with O's label) plus J_o over the
 *      observed points inside V(O) (R10) and inside no volume of S's
 *      objects, each tested against the points R \ C of the composed render
 *      (every object's own points, R6 with each object's own label), as
 *      Eq. 3 and Eq. 4 with R8-R9.  An edge from the root is the plain score.
 *   M4 A state's cost is the sum of its edge costs; a goal's J_r part is the
 *      J_r of the composed scene, since no pixel changes owner down a path.
 *      The search keeps, level by level, the B states of least (cost,
 *      sequence), sequences compared lexicographically as (object, pose
 *      index) pairs, and expands each into all its monotone successors; it
 *      returns the goal of least (cost, sequence).  When B is at least the
 *      size of every level the search is exhaustive and returns the
 *      least-cost goal of the whole tree.
 *   M5 Nearest-neighbour marking of J_o (R12) is not combined with the tree.
 *
 * Colour: sRGB8 is linearised with the IEC 61966-2-1 piecewise curve (256-
 * entry table computed in binary64), mapped to XYZ with the four-digit sRGB
 * matrix, and to CIELAB with the white point equal to the matrix row sums
 * (so sRGB white maps to L* = 100, a* = b* = 0).  CIEDE2000 uses
 * kL = kC = kH = 1.  Parity unpinned: the rotation term R_T, the phase
 * offsets of the hue weighting T (30, 6 and 63 degrees) and the branch that
 * wraps the mean hue across 0/360 degrees.  The tests pin CIEDE2000 only
 * where these vanish or cancel (neutral colours, pure chroma on a*, mirror
 * hue pairs, symmetry), and no published table of test pairs is at hand.
 *
 * Search: the counts are defined by brute force (each point against the
 * whole other cloud).  oracle_score_windowed reaches the same counts by
 * scanning only the pixels of a window that provably holds every neighbour
 * (or_window); the tests pin it equal to brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_USE_RGB 1u
#define OR_MARK_OCCLUDERS 2u
#define OR_VOL_MASK (3u << 4)
#define OR_VOL_AABB (0u << 4)
#define OR_VOL_CYL (1u << 4)
#define OR_VOL_LABEL (2u << 4)
#define OR_JO_NN (1u << 6)

#define OR_NEAR_MM 100.0
#define OR_COORD_LIMIT 16777216.0
#define OR_EMPTY_KEY 0xFFFFFFFFu

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
} oracle_intrinsics;

typedef struct {
    const float *xyz;     /* n_verts * 3, millimetres, object frame */
    int32_t n_verts;
    const int32_t *tri;   /* n_tris * 3 */
    int32_t n_tris;
    const uint8_t *rgb;   /* n_verts * 3 sRGB8, or NULL */
} oracle_mesh;

typedef struct {
    oracle_intrinsics K;
    const uint16_t *depth;  /* H * W millimetres, 0 = no reading */
    const uint8_t *rgb;     /* H * W * 3 sRGB8, or NULL */
    const int32_t *labels;  /* H * W, or NULL */
    float delta_mm;
    float tau_c;
    uint32_t flags;
    int32_t stride;
} oracle_scene;

/* ------------------------------------------------------------------ */
/* Geometry                                                           */
/* ------------------------------------------------------------------ */

typedef struct {
    int ok;          /* 1 if the vertex may take part in a drawn triangle */
    int32_t U, V;    /* 24.8 fixed point screen position */
    double iz;       /* 1 / Zc */
} or_vertex;

static void or_transform(const float *pose, const float *v, double out[3])
{
    double x = (double)v[0], y = (double)v[1], z = (double)v[2];
    out[0] = (((double)pose[0] * x + (double)pose[1] * y) + (double)pose[2] * z) + (double)pose[3];
    out[1] = (((double)pose[4] * x + (double)pose[5] * y) + (double)pose[6] * z) + (double)pose[7];
    out[2] = (((double)pose[8] * x + (double)pose[9] * y) + (double)pose[10] * z) + (double)pose[11];
}

static or_vertex or_project(const float *pose, const float *v, const oracle_intrinsics *K)
{
    or_vertex o;
    double c[3];
    or_transform(pose, v, c);
    o.ok = 0; o.U = 0; o.V = 0; o.iz = 0.0;
    if (!(c[2] >= OR_NEAR_MM)) return o;
    o.iz = 1.0 / c[2];
    double u = (((double)K->fx * c[0]) * o.iz) + (double)K->cx;
    double w = (((double)K->fy * c[1]) * o.iz) + (double)K->cy;
    double su = 256.0 * u, sv = 256.0 * w;
    if (!(fabs(su) <= OR_COORD_LIMIT) || !(fabs(sv) <= OR_COORD_LIMIT)) return o;
    o.U = (int32_t)nearbyint(su);
    o.V = (int32_t)nearbyint(sv);
    o.ok = 1;
    return o;
}

static int64_t or_edge(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py)
{
    return (by - ay) * (px - ax) - (bx - ax) * (py - ay);
}

static int or_top_left(int64_t ax, int64_t ay, int64_t bx, int64_t by)
{
    int64_t dy = by - ay, dx = bx - ax;
    return dy > 0 || (dy == 0 && dx < 0);
}

static int or_inside(int64_t e, int tl) { return e > 0 || (e == 0 && tl); }

static int32_t or_floor_div256(int64_t a) { return (int32_t)(a >= 0 ? a / 256 : -((-a + 255) / 256)); }
static int32_t or_ceil_div256(int64_t a) { return (int32_t)(a >= 0 ? (a + 255) / 256 : -((-a) / 256)); }

/* Render one pose of one mesh into full-size images.  depth: 0 where empty.
 * tri_id: winning triangle or -1.  rgb (optional, needs mesh colours). */
int oracle_render(const oracle_mesh *m, const float *pose, const oracle_intrinsics *K,
                  uint16_t *depth, int32_t *tri_id, uint8_t *rgb)
{
    const int W = K->width, H = K->height;
    if (W <= 0 || H <= 0 || m->n_tris > 65536 || m->n_verts <= 0) return -1;
    uint32_t *zbuf = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)W * H);
    or_vertex *pv = (or_vertex *)malloc(sizeof(or_vertex) * (size_t)m->n_verts);
    if (!zbuf || !pv) { free(zbuf); free(pv); return -2; }
    for (size_t k = 0; k < (size_t)W * H; ++k) zbuf[k] = OR_EMPTY_KEY;
    for (int32_t k = 0; k < m->n_verts; ++k) pv[k] = or_project(pose, m->xyz + 3 * (size_t)k, K);

    for (int32_t t = 0; t < m->n_tris; ++t) {
        const int32_t *ix = m->tri + 3 * (size_t)t;
        const or_vertex a = pv[ix[0]], b = pv[ix[1]], c = pv[ix[2]];
        if (!a.ok || !b.ok || !c.ok) continue;
        int64_t A = or_edge(a.U, a.V, b.U, b.V, c.U, c.V);
        if (A <= 0) continue;
        int64_t minU = a.U, maxU = a.U, minV = a.V, maxV = a.V;
        if (b.U < minU) minU = b.U; if (b.U > maxU) maxU = b.U;
        if (c.U < minU) minU = c.U; if (c.U > maxU) maxU = c.U;
        if (b.V < minV) minV = b.V; if (b.V > maxV) maxV = b.V;
        if (c.V < minV) minV = c.V; if (c.V > maxV) maxV = c.V;
        int32_t i0 = or_ceil_div256(minU), i1 = or_floor_div256(maxU);
        int32_t j0 = or_ceil_div256(minV), j1 = or_floor_div256(maxV);
        if (i0 < 0) i0 = 0;
        if (j0 < 0) j0 = 0;
        if (i1 > W - 1) i1 = W - 1;
        if (j1 > H - 1) j1 = H - 1;
        int tl0 = or_top_left(b.U, b.V, c.U, c.V);
        int tl1 = or_top_left(c.U, c.V, a.U, a.V);
        int tl2 = or_top_left(a.U, a.V, b.U, b.V);
        for (int32_t j = j0; j <= j1; ++j) {
            for (int32_t i = i0; i <= i1; ++i) {
                int64_t px = 256 * (int64_t)i, py = 256 * (int64_t)j;
                int64_t w0 = or_edge(b.U, b.V, c.U, c.V, px, py);
                int64_t w1 = or_edge(c.U, c.V, a.U, a.V, px, py);
                int64_t w2 = or_edge(a.U, a.V, b.U, b.V, px, py);
                if (!or_inside(w0, tl0) || !or_inside(w1, tl1) || !or_inside(w2, tl2)) continue;
                double t0 = (double)w0 * a.iz, t1 = (double)w1 * b.iz, t2 = (double)w2 * c.iz;
                double s = (t0 + t1) + t2;
                double z = (double)A / s;
                double d = nearbyint(z);
                if (!(d >= 1.0 && d <= 65534.0)) continue;
                uint32_t key = ((uint32_t)d << 16) | (uint32_t)t;
                size_t k = (size_t)j * W + i;
                if (key < zbuf[k]) zbuf[k] = key;
            }
        }
    }

    for (int32_t j = 0; j < H; ++j) {
        for (int32_t i = 0; i < W; ++i) {
            size_t k = (size_t)j * W + i;
            uint32_t key = zbuf[k];
            if (key == OR_EMPTY_KEY) {
                depth[k] = 0;
                if (tri_id) tri_id[k] = -1;
                if (rgb) rgb[3 * k] = rgb[3 * k + 1] = rgb[3 * k + 2] = 0;
                continue;
            }
            if (rgb && !m->rgb) {
                rgb[3 * k] = rgb[3 * k + 1] = rgb[3 * k + 2] = 0;
            }
            int32_t t = (int32_t)(key & 0xFFFFu);
            depth[k] = (uint16_t)(key >> 16);
            if (tri_id) tri_id[k] = t;
            if (rgb && m->rgb) {
                const int32_t *ix = m->tri + 3 * (size_t)t;
                const or_vertex a = pv[ix[0]], b = pv[ix[1]], c = pv[ix[2]];
                int64_t px = 256 * (int64_t)i, py = 256 * (int64_t)j;
                int64_t w0 = or_edge(b.U, b.V, c.U, c.V, px, py);
                int64_t w1 = or_edge(c.U, c.V, a.U, a.V, px, py);
                int64_t w2 = or_edge(a.U, a.V, b.U, b.V, px, py);
                double t0 = (double)w0 * a.iz, t1 = (double)w1 * b.iz, t2 = (double)w2 * c.iz;
                double s = (t0 + t1) + t2;
                for (int ch = 0; ch < 3; ++ch) {
                    double c0 = m->rgb[3 * (size_t)ix[0] + ch];
                    double c1 = m->rgb[3 * (size_t)ix[1] + ch];
                    double c2 = m->rgb[3 * (size_t)ix[2] + ch];
                    double v = nearbyint(((t0 * c0 + t1 * c1) + t2 * c2) / s);
                    if (v < 0.0) v = 0.0;
                    if (v > 255.0) v = 255.0;
                    rgb[3 * k + ch] = (uint8_t)v;
                }
            }
        }
    }
    free(zbuf);
    free(pv);
    return 0;
}

/* Back-projection of pixel (i, j) at depth d mm to a point in 1/16 mm. */
void oracle_backproject(const oracle_intrinsics *K, int32_t i, int32_t j, int32_t d, int32_t out[3])
{
    double kx = (((double)i - (double)K->cx) * 16.0) / (double)K->fx;
    double ky = (((double)j - (double)K->cy) * 16.0) / (double)K->fy;
    out[0] = (int32_t)nearbyint(kx * (double)d);
    out[1] = (int32_t)nearbyint(ky * (double)d);
    out[2] = 16 * d;
}

/* ------------------------------------------------------------------ */
/* Colour: sRGB8 -> CIELAB, CIEDE2000                                  */
/* ------------------------------------------------------------------ */

static double or_srgb_linear64(int v)
{
    double c = (double)v / 255.0;
    return c <= 0.04045 ? c / 12.92 : pow((c + 0.055) / 1.055, 2.4);
}

static double or_lab_f64(double t)
{
    const double e = (6.0 / 29.0) * (6.0 / 29.0) * (6.0 / 29.0);
    return t > e ? cbrt(t) : t / (3.0 * (6.0 / 29.0) * (6.0 / 29.0)) + 4.0 / 29.0;
}

void oracle_srgb_to_lab64(const uint8_t *rgb, double *lab)
{
    double r = or_srgb_linear64(rgb[0]), g = or_srgb_linear64(rgb[1]), b = or_srgb_linear64(rgb[2]);
    double X = (0.4124 * r + 0.3576 * g) + 0.1805 * b;
    double Y = (0.2126 * r + 0.7152 * g) + 0.0722 * b;
    double Z = (0.0193 * r + 0.1192 * g) + 0.9505 * b;
    double Xn = (0.4124 + 0.3576) + 0.1805;
    double Yn = (0.2126 + 0.7152) + 0.0722;
    double Zn = (0.0193 + 0.1192) + 0.9505;
    double fx = or_lab_f64(X / Xn), fy = or_lab_f64(Y / Yn), fz = or_lab_f64(Z / Zn);
    lab[0] = 116.0 * fy - 16.0;
    lab[1] = 500.0 * (fx - fy);
    lab[2] = 200.0 * (fy - fz);
}

double oracle_ciede2000_64(const double *x, const double *y)
{
    const double PI = 3.14159265358979323846;
    const double D2R = PI / 180.0, R2D = 180.0 / PI;
    const double P25 = 6103515625.0; /* 25^7 */
    double L1 = x[0], a1 = x[1], b1 = x[2];
    double L2 = y[0], a2 = y[1], b2 = y[2];
    double C1 = sqrt(a1 * a1 + b1 * b1), C2 = sqrt(a2 * a2 + b2 * b2);
    double Cm = (C1 + C2) / 2.0;
    double Cm7 = Cm * Cm * Cm * Cm * Cm * Cm * Cm;
    double G = 0.5 * (1.0 - sqrt(Cm7 / (Cm7 + P25)));
    double a1p = (1.0 + G) * a1, a2p = (1.0 + G) * a2;
    double C1p = sqrt(a1p * a1p + b1 * b1), C2p = sqrt(a2p * a2p + b2 * b2);
    double h1p = (a1p == 0.0 && b1 == 0.0) ? 0.0 : atan2(b1, a1p) * R2D;
    double h2p = (a2p == 0.0 && b2 == 0.0) ? 0.0 : atan2(b2, a2p) * R2D;
    if (h1p < 0.0) h1p += 360.0;
    if (h2p < 0.0) h2p += 360.0;
    double dLp = L2 - L1;
    double dCp = C2p - C1p;
    double dhp;
    double CC = C1p * C2p;
    if (CC == 0.0) dhp = 0.0;
    else if (fabs(h2p - h1p) <= 180.0) dhp = h2p - h1p;
    else if (h2p - h1p > 180.0) dhp = h2p - h1p - 360.0;
    else dhp = h2p - h1p + 360.0;
    double dHp = 2.0 * sqrt(CC) * sin(dhp * D2R / 2.0);
    double Lmp = (L1 + L2) / 2.0;
    double Cmp = (C1p + C2p) / 2.0;
    double hmp;
    if (CC == 0.0) hmp = h1p + h2p;
    else if (fabs(h1p - h2p) <= 180.0) hmp = (h1p + h2p) / 2.0;
    else if (h1p + h2p < 360.0) hmp = (h1p + h2p + 360.0) / 2.0;
    else hmp = (h1p + h2p - 360.0) / 2.0;
    double T = 1.0 - 0.17 * cos((hmp - 30.0) * D2R) + 0.24 * cos(2.0 * hmp * D2R)
               + 0.32 * cos((3.0 * hmp + 6.0) * D2R) - 0.20 * cos((4.0 * hmp - 63.0) * D2R);
    double dth = 30.0 * exp(-((hmp - 275.0) / 25.0) * ((hmp - 275.0) / 25.0));
    double Cmp7 = Cmp * Cmp * Cmp * Cmp * Cmp * Cmp * Cmp;
    double RC = 2.0 * sqrt(Cmp7 / (Cmp7 + P25));
    double Lm50 = (Lmp - 50.0) * (Lmp - 50.0);
    double SL = 1.0 + 0.015 * Lm50 / sqrt(20.0 + Lm50);
    double SC = 1.0 + 0.045 * Cmp;
    double SH = 1.0 + 0.015 * Cmp * T;
    double RT = -sin(2.0 * dth * D2R) * RC;
    double tL = dLp / SL, tC = dCp / SC, tH = dHp / SH;
    return sqrt(tL * tL + tC * tC + tH * tH + RT * tC * tH);
}

/* binary32 twins: the precision in which the colour decision is taken. */
static float or_lin32_table[256];
static int or_lin32_ready = 0;

static void or_lin32_init(void)
{
    if (or_lin32_ready) return;
    for (int v = 0; v < 256; ++v) or_lin32_table[v] = (float)or_srgb_linear64(v);
    or_lin32_ready = 1;
}

static float or_lab_f32(float t)
{
    const float e = 216.0f / 24389.0f;          /* (6/29)^3 */
    const float k = 841.0f / 108.0f;            /* 1 / (3 (6/29)^2) */
    return t > e ? cbrtf(t) : t * k + 4.0f / 29.0f;
}

void oracle_srgb_to_lab32(const uint8_t *rgb, float *lab)
{
    or_lin32_init();
    float r = or_lin32_table[rgb[0]], g = or_lin32_table[rgb[1]], b = or_lin32_table[rgb[2]];
    float X = (0.4124f * r + 0.3576f * g) + 0.1805f * b;
    float Y = (0.2126f * r + 0.7152f * g) + 0.0722f * b;
    float Z = (0.0193f * r + 0.1192f * g) + 0.9505f * b;
    float Xn = (0.4124f + 0.3576f) + 0.1805f;
    float Yn = (0.2126f + 0.7152f) + 0.0722f;
    float Zn = (0.0193f + 0.1192f) + 0.9505f;
    float fx = or_lab_f32(X / Xn), fy = or_lab_f32(Y / Yn), fz = or_lab_f32(Z / Zn);
    lab[0] = 116.0f * fy - 16.0f;
    lab[1] = 500.0f * (fx - fy);
    lab[2] = 200.0f * (fy - fz);
}

float oracle_ciede2000_32(const float *x, const float *y)
{
    const float D2R = 0.017453292519943295f, R2D = 57.29577951308232f;
    const float P25 = 6103515625.0f;
    float L1 = x[0], a1 = x[1], b1 = x[2];
    float L2 = y[0], a2 = y[1], b2 = y[2];
    float C1 = sqrtf(a1 * a1 + b1 * b1), C2 = sqrtf(a2 * a2 + b2 * b2);
    float Cm = (C1 + C2) * 0.5f;
    float Cm2 = Cm * Cm;
    float Cm7 = ((Cm2 * Cm2) * Cm2) * Cm;
    float G = 0.5f * (1.0f - sqrtf(Cm7 / (Cm7 + P25)));
    float a1p = (1.0f + G) * a1, a2p = (1.0f + G) * a2;
    float C1p = sqrtf(a1p * a1p + b1 * b1), C2p = sqrtf(a2p * a2p + b2 * b2);
    float h1p = (a1p == 0.0f && b1 == 0.0f) ? 0.0f : atan2f(b1, a1p) * R2D;
    float h2p = (a2p == 0.0f && b2 == 0.0f) ? 0.0f : atan2f(b2, a2p) * R2D;
    if (h1p < 0.0f) h1p += 360.0f;
    if (h2p < 0.0f) h2p += 360.0f;
    float dLp = L2 - L1;
    float dCp = C2p - C1p;
    float CC = C1p * C2p;
    float dhp;
    if (CC == 0.0f) dhp = 0.0f;
    else if (fabsf(h2p - h1p) <= 180.0f) dhp = h2p - h1p;
    else if (h2p - h1p > 180.0f) dhp = h2p - h1p - 360.0f;
    else dhp = h2p - h1p + 360.0f;
    float dHp = 2.0f * sqrtf(CC) * sinf(dhp * D2R * 0.5f);
    float Lmp = (L1 + L2) * 0.5f;
    float Cmp = (C1p + C2p) * 0.5f;
    float hmp;
    if (CC == 0.0f) hmp = h1p + h2p;
    else if (fabsf(h1p - h2p) <= 180.0f) hmp = (h1p + h2p) * 0.5f;
    else if (h1p + h2p < 360.0f) hmp = (h1p + h2p + 360.0f) * 0.5f;
    else hmp = (h1p + h2p - 360.0f) * 0.5f;
    float T = 1.0f - 0.17f * cosf((hmp - 30.0f) * D2R) + 0.24f * cosf(2.0f * hmp * D2R)
              + 0.32f * cosf((3.0f * hmp + 6.0f) * D2R) - 0.20f * cosf((4.0f * hmp - 63.0f) * D2R);
    float hq = (hmp - 275.0f) / 25.0f;
    float dth = 30.0f * expf(-(hq * hq));
    float Cmp2 = Cmp * Cmp;
    float Cmp7 = ((Cmp2 * Cmp2) * Cmp2) * Cmp;
    float RC = 2.0f * sqrtf(Cmp7 / (Cmp7 + P25));
    float Lm50 = (Lmp - 50.0f) * (Lmp - 50.0f);
    float SL = 1.0f + 0.015f * Lm50 / sqrtf(20.0f + Lm50);
    float SC = 1.0f + 0.045f * Cmp;
    float SH = 1.0f + 0.015f * Cmp * T;
    float RT = -sinf(2.0f * dth * D2R) * RC;
    float tL = dLp / SL, tC = dCp / SC, tH = dHp / SH;
    return sqrtf(tL * tL + tC * tC + tH * tH + RT * tC * tH);
}

/* ------------------------------------------------------------------ */
/* Cost (Eq. 3 / Eq. 4) by brute force                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    int32_t *x, *y, *z, *pix;
    float *lab; /* n * 3, RGB mode only */
} or_cloud;

static void or_cloud_free(or_cloud *c)
{
    free(c->x); free(c->y); free(c->z); free(c->pix); free(c->lab);
    memset(c, 0, sizeof(*c));
}

static int or_cloud_alloc(or_cloud *c, size_t n, int with_lab)
{
    memset(c, 0, sizeof(*c));
    size_t m = n ? n : 1;
    c->x = (int32_t *)malloc(m * sizeof(int32_t));
    c->y = (int32_t *)malloc(m * sizeof(int32_t));
    c->z = (int32_t *)malloc(m * sizeof(int32_t));
    c->pix = (int32_t *)malloc(m * sizeof(int32_t));
    c->lab = with_lab ? (float *)malloc(m * 3 * sizeof(float)) : NULL;
    if (!c->x || !c->y || !c->z || !c->pix || (with_lab && !c->lab)) { or_cloud_free(c); return -1; }
    return 0;
}

/* For point p (coords px,py,pz) search cloud c.  Returns 1 if any point is
 * within dq.  If want_nn, *nn is the index (into c) of the nearest one, ties
 * broken by the lower pixel index. */
static int or_search(const or_cloud *c, int64_t px, int64_t py, int64_t pz, int64_t dq2,
                     int64_t dq, int want_nn, int32_t *nn)
{
    int found = 0;
    int64_t best_d2 = 0;
    int32_t best_pix = 0, best = -1;
    for (int32_t k = 0; k < c->n; ++k) {
        int64_t dz = (int64_t)c->z[k] - pz;
        if (dz > dq || dz < -dq) continue; /* then dz^2 alone exceeds dq^2 */
        int64_t dx = (int64_t)c->x[k] - px, dy = (int64_t)c->y[k] - py;
        int64_t d2 = dx * dx + dy * dy + dz * dz;
        if (d2 > dq2) continue;
        if (!want_nn) return 1;
        if (!found || d2 < best_d2 || (d2 == best_d2 && c->pix[k] < best_pix)) {
            best_d2 = d2; best_pix = c->pix[k]; best = k;
        }
        found = 1;
    }
    if (nn) *nn = best;
    return found;
}

/* Windowed exact search (a faster route to the same result, for large
 * workloads; the tests pin it equal to or_search).  Every point here is the
 * back-projection of a pixel centre (i, j) at an integer depth Z mm: in exact
 * arithmetic X = (i - cx) Z / fx, and the stored 1/16 mm coordinates differ
 * from the exact ones by at most 1/32 mm per axis.  Two points within dq
 * (1/16 mm units) therefore lie within e = dq/16 + 1/4 mm of each other
 * before rounding.  For such a pair (X, Z), (X', Z') with |X' - X|, |Z' - Z|
 * <= e, Cauchy-Schwarz on (X' - X) Z - X (Z' - Z) gives
 *   |i' - i| = fx |X'/Z' - X/Z| <= fx e sqrt(1 + ((i - cx)/fx)^2) / (Z - e),
 * and likewise for rows with fy, cy.  The window below is that bound's
 * floor plus one pixel (so rounding in binary64 cannot make it too small),
 * or the whole image when Z - e <= 1 mm. */
static void or_window(const oracle_intrinsics *K, int64_t dq, int32_t i, int32_t j, int32_t z_mm, int32_t win[4])
{
    const int W = K->width, H = K->height;
    const double e = (double)dq / 16.0 + 0.25;
    const double den = (double)z_mm - e;
    int32_t wu = W, wv = H;
    if (den > 1.0) {
        const double tx = ((double)i - (double)K->cx) / (double)K->fx;
        const double ty = ((double)j - (double)K->cy) / (double)K->fy;
        const double bu = (double)K->fx * e * sqrt(1.0 + tx * tx) / den;
        const double bv = (double)K->fy * e * sqrt(1.0 + ty * ty) / den;
        if (bu < (double)W) wu = (int32_t)floor(bu) + 1;
        if (bv < (double)H) wv = (int32_t)floor(bv) + 1;
    }
    win[0] = i - wu < 0 ? 0 : i - wu;
    win[1] = i + wu > W - 1 ? W - 1 : i + wu;
    win[2] = j - wv < 0 ? 0 : j - wv;
    win[3] = j + wv > H - 1 ? H - 1 : j + wv;
}

/* or_search restricted to the points of cloud c whose pixels lie in the
 * window win; at[k] is the cloud index of pixel k or -1. */
static int or_search_window(const or_cloud *c, const int32_t *at, int W, const int32_t win[4], int64_t px,
                            int64_t py, int64_t pz, int64_t dq2, int64_t dq, int want_nn, int32_t *nn)
{
    int found = 0;
    int64_t best_d2 = 0;
    int32_t best_pix = 0, best = -1;
    for (int32_t j = win[2]; j <= win[3]; ++j) {
        for (int32_t i = win[0]; i <= win[1]; ++i) {
            const int32_t k = at[(size_t)j * W + i];
            if (k < 0) continue;
            int64_t dz = (int64_t)c->z[k] - pz;
            if (dz > dq || dz < -dq) continue;
            int64_t dx = (int64_t)c->x[k] - px, dy = (int64_t)c->y[k] - py;
            int64_t d2 = dx * dx + dy * dy + dz * dz;
            if (d2 > dq2) continue;
            if (!want_nn) { if (nn) *nn = k; return 1; }
            if (!found || d2 < best_d2 || (d2 == best_d2 && c->pix[k] < best_pix)) {
                best_d2 = d2; best_pix = c->pix[k]; best = k;
            }
            found = 1;
        }
    }
    if (nn) *nn = best;
    return found;
}

/* The object-frame AABB of a mesh. */
static void or_mesh_box(const oracle_mesh *m, double lo[3], double hi[3])
{
    for (int a = 0; a < 3; ++a) { lo[a] = (double)m->xyz[a]; hi[a] = (double)m->xyz[a]; }
    for (int32_t v = 1; v < m->n_verts; ++v)
        for (int a = 0; a < 3; ++a) {
            double c = (double)m->xyz[3 * (size_t)v + a];
            if (c < lo[a]) lo[a] = c;
            if (c > hi[a]) hi[a] = c;
        }
}

/* Is observed point p inside V(O) of the object at `pose` (box lo, hi):
 * its label (label volumes), or the inscribed cylinder or the AABB grown by
 * delta (R10). */
static int or_in_volume(const oracle_scene *sc, int32_t label, const float *pose, const double lo[3],
                        const double hi[3], const or_cloud *obs, int32_t p)
{
    const uint32_t vol = sc->flags & OR_VOL_MASK;
    const double dl = (double)sc->delta_mm;
    if (vol == OR_VOL_LABEL) return sc->labels && sc->labels[obs->pix[p]] == label;
    double e0 = (double)obs->x[p] / 16.0 - (double)pose[3];
    double e1 = (double)obs->y[p] / 16.0 - (double)pose[7];
    double e2 = (double)obs->z[p] / 16.0 - (double)pose[11];
    double q0 = ((double)pose[0] * e0 + (double)pose[4] * e1) + (double)pose[8] * e2;
    double q1 = ((double)pose[1] * e0 + (double)pose[5] * e1) + (double)pose[9] * e2;
    double q2 = ((double)pose[2] * e0 + (double)pose[6] * e1) + (double)pose[10] * e2;
    if (vol == OR_VOL_CYL) {
        double c0 = (lo[0] + hi[0]) / 2.0, c1 = (lo[1] + hi[1]) / 2.0;
        double h0 = (hi[0] - lo[0]) / 2.0, h1 = (hi[1] - lo[1]) / 2.0;
        double rho = (h0 < h1 ? h0 : h1) + dl;
        double a = q0 - c0, b = q1 - c1;
        return (a * a + b * b <= rho * rho) && (lo[2] - dl <= q2) && (q2 <= hi[2] + dl);
    }
    return (lo[0] - dl <= q0) && (q0 <= hi[0] + dl) && (lo[1] - dl <= q1) && (q1 <= hi[1] + dl)
           && (lo[2] - dl <= q2) && (q2 <= hi[2] + dl);
}

/* Score one pose; optionally fill per-pixel detail images:
 *  r_flag[k]: 0 not in R, 1 inlier, 2 outlier (distance), 3 outlier (colour), 4 occluded
 *  o_flag[k]: 0 not in Vset, 1 explained, 2 outlier (distance), 3 outlier (colour) */
static int or_score_one(const oracle_mesh *m, const oracle_scene *sc, int32_t label,
                        const float *pose, const or_cloud *obs, const int32_t *obs_at, int32_t out[4],
                        uint8_t *r_flag, uint8_t *o_flag)
{
    const oracle_intrinsics *K = &sc->K;
    const int W = K->width, H = K->height;
    const size_t N = (size_t)W * H;
    const int use_rgb = (sc->flags & OR_USE_RGB) != 0;
    const int mark = (sc->flags & OR_MARK_OCCLUDERS) != 0;
    const uint32_t vol = sc->flags & OR_VOL_MASK;
    const int nn_mark = (sc->flags & OR_JO_NN) != 0;
    const int64_t dq = (int64_t)nearbyint(16.0 * (double)sc->delta_mm);
    const int64_t dq2 = dq * dq;
    const int stride = sc->stride;
    int rc = 0;

    uint16_t *dren = (uint16_t *)malloc(N * sizeof(uint16_t));
    uint8_t *cren = use_rgb ? (uint8_t *)malloc(N * 3) : NULL;
    uint8_t *marked = nn_mark ? (uint8_t *)calloc(obs->n ? (size_t)obs->n : 1, 1) : NULL;
    int32_t *r_at = obs_at ? (int32_t *)malloc(N * sizeof(int32_t)) : NULL;   /* windowed search: pixel -> R */
    or_cloud R;
    if (!dren || (use_rgb && !cren) || (nn_mark && !marked) || (obs_at && !r_at) || or_cloud_alloc(&R, N, use_rgb)) {
        free(dren); free(cren); free(marked); free(r_at); return -2;
    }
    if (r_at) for (size_t k = 0; k < N; ++k) r_at[k] = -1;
    if (oracle_render(m, pose, K, dren, NULL, cren) != 0) { rc = -1; goto done; }

    /* R \ C : rendered, on the stride grid, not occluded (R6, R7). */
    R.n = 0;
    for (int32_t j = 0; j < H; ++j) {
        for (int32_t i = 0; i < W; ++i) {
            size_t k = (size_t)j * W + i;
            if (r_flag) r_flag[k] = 0;
            int32_t d = dren[k];
            if (d == 0) continue;
            if (i % stride != 0 || j % stride != 0) continue;
            int32_t dob = sc->depth[k];
            if (mark && dob > 0 && 16 * (int64_t)dob + dq < 16 * (int64_t)d) {
                int other = !(vol == OR_VOL_LABEL && sc->labels) || sc->labels[k] != label;
                if (other) { if (r_flag) r_flag[k] = 4; continue; }
            }
            int32_t p[3];
            oracle_backproject(K, i, j, d, p);
            R.x[R.n] = p[0]; R.y[R.n] = p[1]; R.z[R.n] = p[2]; R.pix[R.n] = (int32_t)k;
            if (r_at) r_at[k] = R.n;
            if (use_rgb) oracle_srgb_to_lab32(cren + 3 * k, R.lab + 3 * (size_t)R.n);
            R.n++;
        }
    }

    /* J_r: every rendered point against the whole observed cloud. */
    int32_t jr = 0;
    for (int32_t r = 0; r < R.n; ++r) {
        int32_t nn = -1;
        int found;
        if (obs_at) {
            int32_t win[4];
            or_window(K, dq, R.pix[r] % W, R.pix[r] / W, R.z[r] / 16, win);
            found = or_search_window(obs, obs_at, W, win, R.x[r], R.y[r], R.z[r], dq2, dq, use_rgb || nn_mark, &nn);
        } else {
            found = or_search(obs, R.x[r], R.y[r], R.z[r], dq2, dq, use_rgb || nn_mark, &nn);
        }
        int flag = 1;
        if (!found) flag = 2;
        else if (use_rgb && oracle_ciede2000_32(R.lab + 3 * (size_t)r, obs->lab + 3 * (size_t)nn) > sc->tau_c) flag = 3;
        if (flag != 1) jr++;
        else if (nn_mark) marked[nn] = 1;          /* R12 */
        if (r_flag) r_flag[R.pix[r]] = (uint8_t)flag;
    }

    /* J_o: every observed point inside V(O) against the whole render. */
    double lo[3], hi[3];
    or_mesh_box(m, lo, hi);
    int32_t jo = 0, q = 0;
    for (int32_t p = 0; p < obs->n; ++p) {
        int32_t k = obs->pix[p];
        if (o_flag) o_flag[k] = 0;
        int in = or_in_volume(sc, label, pose, lo, hi, obs, p);
        if (!in) continue;
        q++;
        int flag = 1;
        if (nn_mark) {
            if (!marked[p]) flag = 2;
        } else {
            int32_t nn = -1;
            int found;
            if (obs_at) {
                int32_t win[4];
                or_window(K, dq, k % W, k / W, obs->z[p] / 16, win);
                found = or_search_window(&R, r_at, W, win, obs->x[p], obs->y[p], obs->z[p], dq2, dq, use_rgb, &nn);
            } else {
                found = or_search(&R, obs->x[p], obs->y[p], obs->z[p], dq2, dq, use_rgb, &nn);
            }
            if (!found) flag = 2;
            else if (use_rgb && oracle_ciede2000_32(obs->lab + 3 * (size_t)p, R.lab + 3 * (size_t)nn) > sc->tau_c)
                flag = 3;
        }
        if (flag != 1) jo++;
        if (o_flag) o_flag[k] = (uint8_t)flag;
    }
    out[0] = jr; out[1] = jo; out[2] = R.n; out[3] = q;
done:
    free(dren); free(cren); free(marked); free(r_at); or_cloud_free(&R);
    return rc;
}

static int or_scene_valid(const oracle_mesh *m, const oracle_scene *sc)
{
    if (sc->K.width <= 0 || sc->K.height <= 0 || !sc->depth) return 0;
    if (!(sc->delta_mm > 0.0f) || sc->stride < 1) return 0;
    if ((sc->flags & OR_USE_RGB) && (!sc->rgb || !m->rgb)) return 0;
    uint32_t vol = sc->flags & OR_VOL_MASK;
    if (vol != OR_VOL_AABB && vol != OR_VOL_CYL && vol != OR_VOL_LABEL) return 0;
    if (sc->flags & ~(OR_USE_RGB | OR_MARK_OCCLUDERS | OR_VOL_MASK | OR_JO_NN)) return 0;
    if (vol == OR_VOL_LABEL && !sc->labels) return 0;
    for (int32_t t = 0; t < 3 * m->n_tris; ++t)
        if (m->tri[t] < 0 || m->tri[t] >= m->n_verts) return 0;
    return 1;
}

static int or_observed_cloud(const oracle_scene *sc, or_cloud *obs)
{
    const int W = sc->K.width, H = sc->K.height;
    const int use_rgb = (sc->flags & OR_USE_RGB) != 0;
    size_t n = 0;
    for (size_t k = 0; k < (size_t)W * H; ++k) n += sc->depth[k] > 0;
    if (or_cloud_alloc(obs, n, use_rgb)) return -2;
    obs->n = 0;
    for (int32_t j = 0; j < H; ++j)
        for (int32_t i = 0; i < W; ++i) {
            size_t k = (size_t)j * W + i;
            if (sc->depth[k] == 0) continue;
            int32_t p[3];
            oracle_backproject(&sc->K, i, j, sc->depth[k], p);
            obs->x[obs->n] = p[0]; obs->y[obs->n] = p[1]; obs->z[obs->n] = p[2];
            obs->pix[obs->n] = (int32_t)k;
            if (use_rgb) oracle_srgb_to_lab32(sc->rgb + 3 * k, obs->lab + 3 * (size_t)obs->n);
            obs->n++;
        }
    return 0;
}

/* Threads an OpenMP parallel loop of this library uses by default. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Score n poses over OpenMP threads, by brute force or windowed search. */
static int or_score_many(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *poses,
                         int32_t n, int32_t *jr, int32_t *jo, int32_t *nr, int32_t *nq, int32_t n_threads,
                         int windowed)
{
    if (n < 0 || !or_scene_valid(m, sc) || m->n_tris > 65536) return -1;
    or_lin32_init();
    or_cloud obs;
    if (or_observed_cloud(sc, &obs)) return -2;
    int32_t *obs_at = NULL;
    if (windowed) {
        const size_t N = (size_t)sc->K.width * sc->K.height;
        obs_at = (int32_t *)malloc(N * sizeof(int32_t));
        if (!obs_at) { or_cloud_free(&obs); return -2; }
        for (size_t k = 0; k < N; ++k) obs_at[k] = -1;
        for (int32_t p = 0; p < obs.n; ++p) obs_at[obs.pix[p]] = p;
    }
    int err = 0;
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(| : err)
#endif
    for (int32_t p = 0; p < n; ++p) {
        int32_t out[4] = {0, 0, 0, 0};
        int rc = or_score_one(m, sc, label, poses + 12 * (size_t)p, &obs, obs_at, out, NULL, NULL);
        if (rc) err |= 1;
        jr[p] = out[0]; jo[p] = out[1];
        if (nr) nr[p] = out[2];
        if (nq) nq[p] = out[3];
    }
    (void)n_threads;
    free(obs_at);
    or_cloud_free(&obs);
    return err ? -2 : 0;
}

/* Score n poses by brute force (n x 12 binary32, row-major [R|t], object ->
 * camera, mm).  Outputs jr, jo, nr (= L, the size of R \ C) and nq (= Q, the
 * size of the observed set inside V).  n_threads <= 0 uses the OpenMP
 * default. */
int oracle_score(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *poses,
                 int32_t n, int32_t *jr, int32_t *jo, int32_t *nr, int32_t *nq, int32_t n_threads)
{
    return or_score_many(m, sc, label, poses, n, jr, jo, nr, nq, n_threads, 0);
}

/* The same counts by the windowed exact search (or_window): each point is
 * compared only with the other cloud's points whose pixels lie within the
 * window that provably contains all its neighbours. */
int oracle_score_windowed(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *poses,
                          int32_t n, int32_t *jr, int32_t *jo, int32_t *nr, int32_t *nq, int32_t n_threads)
{
    return or_score_many(m, sc, label, poses, n, jr, jo, nr, nq, n_threads, 1);
}

/* One pose, with per-pixel classification images (see or_score_one). */
static int or_detail(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *pose,
                     int32_t out[4], uint8_t *r_flag, uint8_t *o_flag, int windowed)
{
    if (!or_scene_valid(m, sc) || m->n_tris > 65536) return -1;
    or_lin32_init();
    or_cloud obs;
    if (or_observed_cloud(sc, &obs)) return -2;
    size_t N = (size_t)sc->K.width * sc->K.height;
    int32_t *obs_at = NULL;
    if (windowed) {
        obs_at = (int32_t *)malloc(N * sizeof(int32_t));
        if (!obs_at) { or_cloud_free(&obs); return -2; }
        for (size_t k = 0; k < N; ++k) obs_at[k] = -1;
        for (int32_t p = 0; p < obs.n; ++p) obs_at[obs.pix[p]] = p;
    }
    if (o_flag) memset(o_flag, 0, N);
    int rc = or_score_one(m, sc, label, pose, &obs, obs_at, out, r_flag, o_flag);
    free(obs_at);
    or_cloud_free(&obs);
    return rc;
}

/* One pose, with per-pixel classification images (see or_score_one), by
 * brute force. */
int oracle_score_detail(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *pose,
                        int32_t out[4], uint8_t *r_flag, uint8_t *o_flag)
{
    return or_detail(m, sc, label, pose, out, r_flag, o_flag, 0);
}

/* The same by the windowed exact search. */
int oracle_score_detail_windowed(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *pose,
                                 int32_t out[4], uint8_t *r_flag, uint8_t *o_flag)
{
    return or_detail(m, sc, label, pose, out, r_flag, o_flag, 1);
}

/* ------------------------------------------------------------------ */
/* ICP refinement (readings I1-I8)                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n, sq[3], sc[3], sqq[3][3], sqc[3][3];
} or_icp_sums;

static void or_icp_add(or_icp_sums *z, const int64_t q[3], const int64_t c[3])
{
    z->n++;
    for (int a = 0; a < 3; ++a) {
        z->sq[a] += q[a];
        z->sc[a] += c[a];
        for (int b = 0; b < 3; ++b) {
            z->sqq[a][b] += q[a] * q[b];
            z->sqc[a][b] += q[a] * c[b];
        }
    }
}

/* q = rint(A s + b) (I2). */
static void or_icp_map(const double A[9], const double b[3], const int32_t s[3], int64_t q[3])
{
    for (int a = 0; a < 3; ++a) {
        double v = ((A[3 * a] * (double)s[0] + A[3 * a + 1] * (double)s[1]) + A[3 * a + 2] * (double)s[2]) + b[a];
        q[a] = (int64_t)nearbyint(v);
    }
}

/* One update from the sums (I4-I6): composes the increment into (A, b).
 * Returns 0, or 1 when the 6-DoF system is singular (nothing changes). */
static int or_icp_update(const or_icp_sums *z, int dof, const double u[3], double A[9], double b[3])
{
    const double n = (double)z->n;
    double mq[3], mc[3], S[3][3], H[3][3];
    for (int a = 0; a < 3; ++a) {
        mq[a] = (double)z->sq[a] / n;
        mc[a] = (double)z->sc[a] / n;
    }
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            S[a][c] = (double)z->sqq[a][c] - ((double)z->sq[a] * (double)z->sq[c]) / n;
            H[a][c] = (double)z->sqc[a][c] - ((double)z->sq[a] * (double)z->sc[c]) / n;
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
        if (h > 0.0) { co = Ap / h; si = B / h; }
        const double K[3][3] = {{0.0, -u[2], u[1]}, {u[2], 0.0, -u[0]}, {-u[1], u[0], 0.0}};
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                R[a][c] = ((a == c ? co : 0.0) + si * K[a][c]) + ((1.0 - co) * u[a]) * u[c];
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
        for (int a = 0; a < 3; ++a)
            h[a] = (((adj[a][0] * w[0] + adj[a][1] * w[1]) + adj[a][2] * w[2]) / det) / 2.0;
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
    memcpy(A, An, sizeof(An));
    memcpy(b, bn, sizeof(bn));
    return 0;
}

/* The object z axis of a pose, normalised (I5, 3-DoF). */
static void or_pose_axis(const float *pose, double u[3])
{
    const double v[3] = {(double)pose[2], (double)pose[6], (double)pose[10]};
    const double nrm = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    for (int a = 0; a < 3; ++a) u[a] = v[a] / nrm;
}

/* The refined pose (I8). */
static void or_icp_pose(const float *pose, const double A[9], const double b[3], float *out)
{
    for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c)
            out[4 * a + c] = (float)((A[3 * a] * (double)pose[c] + A[3 * a + 1] * (double)pose[4 + c])
                                     + A[3 * a + 2] * (double)pose[8 + c]);
        const double t = ((A[3 * a] * (16.0 * (double)pose[3]) + A[3 * a + 1] * (16.0 * (double)pose[7]))
                          + A[3 * a + 2] * (16.0 * (double)pose[11])) + b[a];
        out[4 * a + 3] = (float)(t / 16.0);
    }
}

/* ICP of one pose against the observed cloud (I1-I8). */
static int or_icp_one(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *pose,
                      const or_cloud *obs, double rho, int32_t iterations, int32_t stride, int32_t dof,
                      int32_t min_points, float *out, int32_t *iters_out, int32_t *matched_out)
{
    const oracle_intrinsics *K = &sc->K;
    const int W = K->width, H = K->height;
    const size_t N = (size_t)W * H;
    const int mark = (sc->flags & OR_MARK_OCCLUDERS) != 0;
    const uint32_t vol = sc->flags & OR_VOL_MASK;
    const int64_t dq = (int64_t)nearbyint(16.0 * (double)sc->delta_mm);
    const int64_t rq = (int64_t)nearbyint(16.0 * rho);
    const int64_t rq2 = rq * rq;
    uint16_t *dren = (uint16_t *)malloc(N * sizeof(uint16_t));
    int32_t *src = (int32_t *)malloc(3 * N * sizeof(int32_t));
    int64_t *qprev = (int64_t *)malloc(3 * N * sizeof(int64_t));
    int64_t *qcur = (int64_t *)malloc(3 * N * sizeof(int64_t));
    int rc = 0;
    if (!dren || !src || !qprev || !qcur) { rc = -2; goto done; }
    if (oracle_render(m, pose, K, dren, NULL, NULL) != 0) { rc = -1; goto done; }

    /* I1: the source cloud */
    size_t ns = 0;
    for (int32_t j = 0; j < H; ++j)
        for (int32_t i = 0; i < W; ++i) {
            size_t k = (size_t)j * W + i;
            int32_t d = dren[k];
            if (d == 0 || i % stride != 0 || j % stride != 0) continue;
            int32_t dob = sc->depth[k];
            if (mark && dob > 0 && 16 * (int64_t)dob + dq < 16 * (int64_t)d) {
                int other = !(vol == OR_VOL_LABEL && sc->labels) || sc->labels[k] != label;
                if (other) continue;
            }
            oracle_backproject(K, i, j, d, src + 3 * ns);
            ns++;
        }

    double A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, b[3] = {0, 0, 0}, u[3];
    or_pose_axis(pose, u);
    int32_t iters = 0, matched = 0;
    for (int32_t k = 0; k < iterations; ++k) {
        for (size_t p = 0; p < ns; ++p) or_icp_map(A, b, src + 3 * p, qcur + 3 * p);
        if (k > 0 && memcmp(qcur, qprev, 3 * ns * sizeof(int64_t)) == 0) break;   /* I7 */
        or_icp_sums z;
        memset(&z, 0, sizeof(z));
        for (size_t p = 0; p < ns; ++p) {
            const int64_t *q = qcur + 3 * p;
            int64_t best_d2 = 0;
            int32_t best = -1;
            for (int32_t t = 0; t < obs->n; ++t) {   /* I3: brute force, pixel order */
                int64_t dx = (int64_t)obs->x[t] - q[0], dy = (int64_t)obs->y[t] - q[1], dz = (int64_t)obs->z[t] - q[2];
                int64_t d2 = dx * dx + dy * dy + dz * dz;
                if (d2 <= rq2 && (best < 0 || d2 < best_d2)) { best_d2 = d2; best = t; }
            }
            if (best >= 0) {
                const int64_t c[3] = {obs->x[best], obs->y[best], obs->z[best]};
                or_icp_add(&z, q, c);
            }
        }
        matched = (int32_t)z.n;
        if (z.n < min_points) break;
        if (or_icp_update(&z, dof, u, A, b)) break;
        iters = k + 1;
        int64_t *tmp = qprev; qprev = qcur; qcur = tmp;
    }
    or_icp_pose(pose, A, b, out);
    *iters_out = iters;
    *matched_out = matched;
done:
    free(dren); free(src); free(qprev); free(qcur);
    return rc;
}

/* G1: the integer normal direction c of the point at pixel (i, j); 0 when
 * there is none. */
static int or_normal(const uint16_t *depth, const oracle_intrinsics *K, int32_t i, int32_t j, int32_t gap,
                     int64_t c[3])
{
    const int W = K->width, H = K->height;
    if (i < 1 || j < 1 || i > W - 2 || j > H - 2) return 0;
    const int32_t d = depth[(size_t)j * W + i];
    const int32_t nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
    int32_t p[4][3];
    for (int k = 0; k < 4; ++k) {
        const int32_t dn = depth[(size_t)nb[k][1] * W + nb[k][0]];
        if (d == 0 || dn == 0 || dn - d > gap || d - dn > gap) return 0;
        oracle_backproject(K, nb[k][0], nb[k][1], dn, p[k]);
    }
    int64_t ex[3], ey[3];
    for (int a = 0; a < 3; ++a) {
        ex[a] = (int64_t)p[1][a] - p[0][a];
        ey[a] = (int64_t)p[3][a] - p[2][a];
        if (ex[a] > 16384 || ex[a] < -16384 || ey[a] > 16384 || ey[a] < -16384) return 0;
    }
    c[0] = ex[1] * ey[2] - ex[2] * ey[1];
    c[1] = ex[2] * ey[0] - ex[0] * ey[2];
    c[2] = ex[0] * ey[1] - ex[1] * ey[0];
    return c[0] != 0 || c[1] != 0 || c[2] != 0;
}

static void or_unit(const int64_t c[3], double n[3])
{
    const double x = (double)c[0], y = (double)c[1], z = (double)c[2];
    const double l = sqrt((x * x + y * y) + z * z);
    n[0] = x / l;
    n[1] = y / l;
    n[2] = z / l;
}

/* G4: the 27 fixed-point terms of one match. */
static void or_gicp_terms(const int64_t q[3], const int64_t c[3], const int64_t mu[3], int has_a, const double na[3],
                          int has_b, const double nb[3], const double A[9], uint64_t acc[27])
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
    const double x = (double)(q[0] - mu[0]), y = (double)(q[1] - mu[1]), z = (double)(q[2] - mu[2]);
    const double Kq[3][3] = {{0.0, z, -y}, {-z, 0.0, x}, {y, -x, 0.0}};
    const double e[3] = {(double)(c[0] - q[0]), (double)(c[1] - q[1]), (double)(c[2] - q[2])};
    double MK[3][3], Me[3];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) MK[r][k] = (M[r][0] * Kq[0][k] + M[r][1] * Kq[1][k]) + M[r][2] * Kq[2][k];
        Me[r] = (M[r][0] * e[0] + M[r][1] * e[1]) + M[r][2] * e[2];
    }
    double Hf[6][6];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            Hf[r][k] = (Kq[0][r] * MK[0][k] + Kq[1][r] * MK[1][k]) + Kq[2][r] * MK[2][k];
            Hf[r][3 + k] = MK[k][r];
            Hf[3 + r][3 + k] = M[r][k];
        }
    double g[6];
    for (int r = 0; r < 3; ++r) {
        g[r] = (Kq[0][r] * Me[0] + Kq[1][r] * Me[1]) + Kq[2][r] * Me[2];
        g[3 + r] = Me[r];
    }
    int t = 0;
    for (int r = 0; r < 6; ++r)
        for (int k = r; k < 6; ++k) acc[t++] += (uint64_t)(int64_t)nearbyint(Hf[r][k] * 1024.0);
    for (int r = 0; r < 6; ++r) acc[t++] += (uint64_t)(int64_t)nearbyint(g[r] * 1024.0);
}

/* G5: solve and update; 1 when a pivot fails (nothing changes). */
static int or_gicp_update(const uint64_t acc[27], const int64_t mu[3], double A[9], double b[3])
{
    double Hm[6][6], g[6];
    int t = 0;
    for (int r = 0; r < 6; ++r)
        for (int k = r; k < 6; ++k) {
            Hm[r][k] = (double)(int64_t)acc[t++] / 1024.0;
            Hm[k][r] = Hm[r][k];
        }
    for (int r = 0; r < 6; ++r) g[r] = (double)(int64_t)acc[t++] / 1024.0;
    double L[6][6] = {{0}};
    for (int j = 0; j < 6; ++j) {
        double sjj = Hm[j][j];
        for (int k = 0; k < j; ++k) sjj = sjj - L[j][k] * L[j][k];
        if (!(sjj > 0.0)) return 1;
        L[j][j] = sqrt(sjj);
        for (int i = j + 1; i < 6; ++i) {
            double sij = Hm[i][j];
            for (int k = 0; k < j; ++k) sij = sij - L[i][k] * L[j][k];
            L[i][j] = sij / L[j][j];
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
    memcpy(A, An, sizeof(An));
    memcpy(b, bn, sizeof(bn));
    return 0;
}

/* GICP of one pose (G1-G6). */
static int or_gicp_one(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *pose,
                       const or_cloud *obs, const int64_t *obs_c, const uint8_t *obs_has, double rho,
                       int32_t iterations, int32_t stride, int32_t min_points, float *out, int32_t *iters_out,
                       int32_t *matched_out)
{
    const oracle_intrinsics *K = &sc->K;
    const int W = K->width, H = K->height;
    const size_t N = (size_t)W * H;
    const int mark = (sc->flags & OR_MARK_OCCLUDERS) != 0;
    const uint32_t vol = sc->flags & OR_VOL_MASK;
    const int64_t dq = (int64_t)nearbyint(16.0 * (double)sc->delta_mm);
    const int64_t rq = (int64_t)nearbyint(16.0 * rho);
    const int64_t rq2 = rq * rq;
    const int32_t gap = (int32_t)(rq / 16);
    uint16_t *dren = (uint16_t *)malloc(N * sizeof(uint16_t));
    int32_t *src = (int32_t *)malloc(3 * N * sizeof(int32_t));
    double *srcn = (double *)malloc(3 * N * sizeof(double));
    uint8_t *srch = (uint8_t *)malloc(N);
    int64_t *qprev = (int64_t *)malloc(3 * N * sizeof(int64_t));
    int64_t *qcur = (int64_t *)malloc(3 * N * sizeof(int64_t));
    int32_t *match = (int32_t *)malloc(N * sizeof(int32_t));
    int rc = 0;
    if (!dren || !src || !srcn || !srch || !qprev || !qcur || !match) { rc = -2; goto done; }
    if (oracle_render(m, pose, K, dren, NULL, NULL) != 0) { rc = -1; goto done; }

    size_t ns = 0;
    for (int32_t j = 0; j < H; ++j)
        for (int32_t i = 0; i < W; ++i) {
            size_t k = (size_t)j * W + i;
            int32_t d = dren[k];
            if (d == 0 || i % stride != 0 || j % stride != 0) continue;
            int32_t dob = sc->depth[k];
            if (mark && dob > 0 && 16 * (int64_t)dob + dq < 16 * (int64_t)d) {
                int other = !(vol == OR_VOL_LABEL && sc->labels) || sc->labels[k] != label;
                if (other) continue;
            }
            oracle_backproject(K, i, j, d, src + 3 * ns);
            int64_t c[3];
            srch[ns] = (uint8_t)or_normal(dren, K, i, j, gap, c);
            if (srch[ns]) or_unit(c, srcn + 3 * ns);
            ns++;
        }

    double A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, b[3] = {0, 0, 0};
    int32_t iters = 0, matched = 0;
    for (int32_t k = 0; k < iterations; ++k) {
        for (size_t p = 0; p < ns; ++p) or_icp_map(A, b, src + 3 * p, qcur + 3 * p);
        if (k > 0 && memcmp(qcur, qprev, 3 * ns * sizeof(int64_t)) == 0) break;
        int64_t n = 0, sq[3] = {0, 0, 0};
        for (size_t p = 0; p < ns; ++p) {
            const int64_t *q = qcur + 3 * p;
            int64_t best_d2 = 0;
            int32_t best = -1;
            for (int32_t t = 0; t < obs->n; ++t) {
                int64_t dx = (int64_t)obs->x[t] - q[0], dy = (int64_t)obs->y[t] - q[1], dz = (int64_t)obs->z[t] - q[2];
                int64_t d2 = dx * dx + dy * dy + dz * dz;
                if (d2 <= rq2 && (best < 0 || d2 < best_d2)) { best_d2 = d2; best = t; }
            }
            match[p] = best;
            if (best >= 0) {
                n++;
                for (int a = 0; a < 3; ++a) sq[a] += q[a];
            }
        }
        matched = (int32_t)n;
        if (n < min_points) break;
        int64_t mu[3];
        for (int a = 0; a < 3; ++a) mu[a] = (int64_t)nearbyint((double)sq[a] / (double)n);
        uint64_t acc[27];
        memset(acc, 0, sizeof(acc));
        for (size_t p = 0; p < ns; ++p) {
            if (match[p] < 0) continue;
            const int32_t t = match[p];
            const int64_t c[3] = {obs->x[t], obs->y[t], obs->z[t]};
            double nb[3] = {0.0, 0.0, 0.0};
            if (obs_has[t]) or_unit(obs_c + 3 * (size_t)t, nb);
            or_gicp_terms(qcur + 3 * p, c, mu, srch[p], srcn + 3 * p, obs_has[t], nb, A, acc);
        }
        if (or_gicp_update(acc, mu, A, b)) break;
        iters = k + 1;
        int64_t *tmp = qprev; qprev = qcur; qcur = tmp;
    }
    or_icp_pose(pose, A, b, out);
    *iters_out = iters;
    *matched_out = matched;
done:
    free(dren); free(src); free(srcn); free(srch); free(qprev); free(qcur); free(match);
    return rc;
}

/* G1 normals of every pixel of a depth image: H*W*3 binary64 unit vectors,
 * NaN where there is none. */
int oracle_normal_image(const uint16_t *depth, const oracle_intrinsics *K, int32_t gap, double *out)
{
    for (int32_t j = 0; j < K->height; ++j)
        for (int32_t i = 0; i < K->width; ++i) {
            double *o = out + 3 * ((size_t)j * K->width + i);
            int64_t c[3];
            if (or_normal(depth, K, i, j, gap, c)) or_unit(c, o);
            else o[0] = o[1] = o[2] = NAN;
        }
    return 0;
}

/* Plane-to-plane GICP refinement of n poses (G1-G6; 6-DoF).  Arguments as
 * oracle_icp without dof. */
int oracle_gicp(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *poses, int32_t n,
                double rho, int32_t iterations, int32_t stride, int32_t min_points, float *refined, int32_t *iters,
                int32_t *matched, int32_t n_threads)
{
    if (n < 0 || !or_scene_valid(m, sc) || m->n_tris > 65536) return -1;
    if (!(rho > 0.0 && rho <= 100.0) || iterations < 1 || stride < 1 || min_points < 3) return -1;
    or_cloud obs;
    oracle_scene s2 = *sc;
    s2.flags &= ~OR_USE_RGB;
    if (or_observed_cloud(&s2, &obs)) return -2;
    if ((sc->flags & OR_VOL_MASK) == OR_VOL_LABEL) {
        int32_t k = 0;
        for (int32_t t = 0; t < obs.n; ++t) {
            if (sc->labels[obs.pix[t]] != label) continue;
            obs.x[k] = obs.x[t]; obs.y[k] = obs.y[t]; obs.z[k] = obs.z[t]; obs.pix[k] = obs.pix[t];
            k++;
        }
        obs.n = k;
    }
    const int32_t gap = (int32_t)((int64_t)nearbyint(16.0 * rho) / 16);
    int64_t *obs_c = (int64_t *)malloc(3 * (size_t)(obs.n ? obs.n : 1) * sizeof(int64_t));
    uint8_t *obs_has = (uint8_t *)malloc((size_t)(obs.n ? obs.n : 1));
    if (!obs_c || !obs_has) { free(obs_c); free(obs_has); or_cloud_free(&obs); return -2; }
    for (int32_t t = 0; t < obs.n; ++t) {
        const int32_t W = sc->K.width;
        obs_has[t] = (uint8_t)or_normal(sc->depth, &sc->K, obs.pix[t] % W, obs.pix[t] / W, gap, obs_c + 3 * (size_t)t);
    }
    int err = 0;
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(| : err)
#endif
    for (int32_t p = 0; p < n; ++p) {
        if (or_gicp_one(m, sc, label, poses + 12 * (size_t)p, &obs, obs_c, obs_has, rho, iterations, stride,
                        min_points, refined + 12 * (size_t)p, iters + p, matched + p))
            err |= 1;
    }
    (void)n_threads;
    free(obs_c);
    free(obs_has);
    or_cloud_free(&obs);
    return err ? -2 : 0;
}

/* GICP updates on fixed correspondences with given normals (n x 3 binary64
 * unit vectors; has_* flags 0 for none): dst[i] is the match of src[i]. */
int oracle_gicp_pairs(const int32_t *src, const int32_t *dst, const double *src_n, const uint8_t *src_has,
                      const double *dst_n, const uint8_t *dst_has, int32_t n, int32_t iterations, double *A, double *b)
{
    if (n < 3) return -1;
    const double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    memcpy(A, I, sizeof(I));
    b[0] = b[1] = b[2] = 0.0;
    for (int32_t k = 0; k < iterations; ++k) {
        int64_t sq[3] = {0, 0, 0};
        int64_t *qs = (int64_t *)malloc(3 * (size_t)n * sizeof(int64_t));
        if (!qs) return -2;
        for (int32_t p = 0; p < n; ++p) {
            or_icp_map(A, b, src + 3 * (size_t)p, qs + 3 * (size_t)p);
            for (int a = 0; a < 3; ++a) sq[a] += qs[3 * (size_t)p + a];
        }
        int64_t mu[3];
        for (int a = 0; a < 3; ++a) mu[a] = (int64_t)nearbyint((double)sq[a] / (double)n);
        uint64_t acc[27];
        memset(acc, 0, sizeof(acc));
        for (int32_t p = 0; p < n; ++p) {
            const int64_t c[3] = {dst[3 * (size_t)p], dst[3 * (size_t)p + 1], dst[3 * (size_t)p + 2]};
            or_gicp_terms(qs + 3 * (size_t)p, c, mu, src_has[p], src_n + 3 * (size_t)p, dst_has[p], dst_n + 3 * (size_t)p,
                          A, acc);
        }
        free(qs);
        if (or_gicp_update(acc, mu, A, b)) return 1;
    }
    return 0;
}

/* ICP refinement of n poses (readings I1-I8): refined poses (n x 12
 * binary32), the updates applied and the matches of the last iteration
 * examined.  dof is 3 or 6; rho in (0, 100] mm; min_points >= 3. */
int oracle_icp(const oracle_mesh *m, const oracle_scene *sc, int32_t label, const float *poses, int32_t n,
               double rho, int32_t iterations, int32_t stride, int32_t dof, int32_t min_points,
               float *refined, int32_t *iters, int32_t *matched, int32_t n_threads)
{
    if (n < 0 || !or_scene_valid(m, sc) || m->n_tris > 65536) return -1;
    if (!(rho > 0.0 && rho <= 100.0) || iterations < 1 || stride < 1 || (dof != 3 && dof != 6) || min_points < 3)
        return -1;
    or_cloud obs;
    oracle_scene s2 = *sc;
    s2.flags &= ~OR_USE_RGB;
    if (or_observed_cloud(&s2, &obs)) return -2;
    if ((sc->flags & OR_VOL_MASK) == OR_VOL_LABEL) {   /* I1: the object's labelled points only */
        int32_t k = 0;
        for (int32_t t = 0; t < obs.n; ++t) {
            if (sc->labels[obs.pix[t]] != label) continue;
            obs.x[k] = obs.x[t]; obs.y[k] = obs.y[t]; obs.z[k] = obs.z[t]; obs.pix[k] = obs.pix[t];
            k++;
        }
        obs.n = k;
    }
    int err = 0;
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(| : err)
#endif
    for (int32_t p = 0; p < n; ++p) {
        if (or_icp_one(m, sc, label, poses + 12 * (size_t)p, &obs, rho, iterations, stride, dof, min_points,
                       refined + 12 * (size_t)p, iters + p, matched + p))
            err |= 1;
    }
    (void)n_threads;
    or_cloud_free(&obs);
    return err ? -2 : 0;
}

/* The ICP update loop on fixed correspondences: dst[i] is the match of
 * src[i] (n x 3 int32, 1/16 mm); u is the 3-DoF axis.  Runs `iterations`
 * updates (I2, I4-I6) and returns the transform (A row-major, b). */
int oracle_icp_pairs(const int32_t *src, const int32_t *dst, int32_t n, int32_t dof, const double *u,
                     int32_t iterations, double *A, double *b)
{
    if (n < 3 || (dof != 3 && dof != 6)) return -1;
    const double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    memcpy(A, I, sizeof(I));
    b[0] = b[1] = b[2] = 0.0;
    for (int32_t k = 0; k < iterations; ++k) {
        or_icp_sums z;
        memset(&z, 0, sizeof(z));
        for (int32_t p = 0; p < n; ++p) {
            int64_t q[3];
            or_icp_map(A, b, src + 3 * (size_t)p, q);
            const int64_t c[3] = {dst[3 * (size_t)p], dst[3 * (size_t)p + 1], dst[3 * (size_t)p + 2]};
            or_icp_add(&z, q, c);
        }
        if (or_icp_update(&z, dof, u, A, b)) return 1;
    }
    return 0;
}

/* Minimum of J = jr + jo; ties go to the lowest index.  n_ties counts the
 * poses that share the minimum. */
int oracle_best(const int32_t *jr, const int32_t *jo, int32_t n, int32_t *best_idx,
                int32_t *best_cost, int32_t *n_ties)
{
    if (n <= 0) return -1;
    int32_t bi = 0;
    int64_t bc = (int64_t)jr[0] + jo[0];
    int32_t ties = 1;
    for (int32_t p = 1; p < n; ++p) {
        int64_t c = (int64_t)jr[p] + jo[p];
        if (c < bc) { bc = c; bi = p; ties = 1; }
        else if (c == bc) ties++;
    }
    *best_idx = bi;
    *best_cost = (int32_t)bc;
    if (n_ties) *n_ties = ties;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Monotone Scene Generation tree (readings M1-M5)                     */
/* ------------------------------------------------------------------ */

/* M2: compose the renders of a state's objects in order.  depth and own
 * (owner index, -1 none) are W*H, rgb W*H*3 or NULL.  Returns 1 when an
 * object occludes an earlier one (the state is not monotone). */
static int or_compose(const oracle_scene *sc, const oracle_mesh *const *meshes, const float *poses, int32_t n,
                      uint16_t *depth, uint8_t *rgb, int32_t *own)
{
    const size_t N = (size_t)sc->K.width * sc->K.height;
    uint16_t *d = (uint16_t *)malloc(N * sizeof(uint16_t));
    uint8_t *c = rgb ? (uint8_t *)malloc(3 * N) : NULL;
    if (!d || (rgb && !c)) { free(d); free(c); return -2; }
    memset(depth, 0, N * sizeof(uint16_t));
    if (rgb) memset(rgb, 0, 3 * N);
    for (size_t k = 0; k < N; ++k) own[k] = -1;
    int nonmono = 0, rc = 0;
    for (int32_t o = 0; o < n && !rc; ++o) {
        if (oracle_render(meshes[o], poses + 12 * (size_t)o, &sc->K, d, NULL, c) != 0) { rc = -1; break; }
        for (size_t k = 0; k < N; ++k) {
            if (d[k] == 0) continue;
            if (depth[k] > 0) {
                if (d[k] < depth[k]) nonmono = 1;
                continue;
            }
            depth[k] = d[k];
            own[k] = o;
            if (rgb) memcpy(rgb + 3 * k, c + 3 * k, 3);
        }
    }
    free(d); free(c);
    return rc ? rc : nonmono;
}

/* Append pixel k at depth d to cloud R if it is a point of R \ C: on the
 * stride grid and not an occluder (R6 with the owner's label). */
static void or_add_point(const oracle_scene *sc, int32_t label, size_t k, int32_t d, const uint8_t *rgb, or_cloud *R)
{
    const int W = sc->K.width;
    const int32_t i = (int32_t)(k % (size_t)W), j = (int32_t)(k / (size_t)W);
    if (i % sc->stride != 0 || j % sc->stride != 0) return;
    const int64_t dq = (int64_t)nearbyint(16.0 * (double)sc->delta_mm);
    const int32_t dob = sc->depth[k];
    if ((sc->flags & OR_MARK_OCCLUDERS) && dob > 0 && 16 * (int64_t)dob + dq < 16 * (int64_t)d) {
        int other = !((sc->flags & OR_VOL_MASK) == OR_VOL_LABEL && sc->labels) || sc->labels[k] != label;
        if (other) return;
    }
    int32_t p[3];
    oracle_backproject(&sc->K, i, j, d, p);
    R->x[R->n] = p[0]; R->y[R->n] = p[1]; R->z[R->n] = p[2]; R->pix[R->n] = (int32_t)k;
    if (R->lab) oracle_srgb_to_lab32(rgb + 3 * k, R->lab + 3 * (size_t)R->n);
    R->n++;
}

/* M3: the edges from one state (n_state objects: meshes, labels, poses)
 * to object m (label) at each of n poses.  Per pose: valid (M2), jr, jo,
 * nr (|dR \ C|) and nq (observed points charged to the edge); all zero for
 * a successor that is not monotone.  Returns -1 on invalid arguments or a
 * state that is not monotone itself. */
int oracle_msg_expand(const oracle_scene *sc, const oracle_mesh *const *state_meshes, const int32_t *state_labels,
                      const float *state_poses, int32_t n_state, const oracle_mesh *m, int32_t label,
                      const float *poses, int32_t n, int32_t *valid, int32_t *jr, int32_t *jo, int32_t *nr,
                      int32_t *nq, int32_t n_threads)
{
    if (n < 0 || n_state < 0 || !or_scene_valid(m, sc) || m->n_tris > 65536 || (sc->flags & OR_JO_NN)) return -1;
    for (int32_t o = 0; o < n_state; ++o)
        if (!or_scene_valid(state_meshes[o], sc) || state_meshes[o]->n_tris > 65536) return -1;
    or_lin32_init();
    const oracle_intrinsics *K = &sc->K;
    const size_t N = (size_t)K->width * K->height;
    const int use_rgb = (sc->flags & OR_USE_RGB) != 0;
    const int64_t dq = (int64_t)nearbyint(16.0 * (double)sc->delta_mm);
    const int64_t dq2 = dq * dq;
    uint16_t *cd = (uint16_t *)malloc(N * sizeof(uint16_t));
    uint8_t *cc = use_rgb ? (uint8_t *)malloc(3 * N) : NULL;
    int32_t *own = (int32_t *)malloc(N * sizeof(int32_t));
    uint8_t *covered = NULL;
    or_cloud obs, Rs;
    memset(&obs, 0, sizeof(obs));
    memset(&Rs, 0, sizeof(Rs));
    int rc = 0;
    if (!cd || (use_rgb && !cc) || !own || or_observed_cloud(sc, &obs) || or_cloud_alloc(&Rs, N, use_rgb)) {
        rc = -2; goto out;
    }
    rc = or_compose(sc, state_meshes, state_poses, n_state, cd, cc, own);
    if (rc) { rc = rc == 1 ? -1 : rc; goto out; }
    /* the state's own points R_S \ C, and the observed points inside some
     * volume of the state's objects */
    Rs.n = 0;
    for (size_t k = 0; k < N; ++k)
        if (cd[k] > 0) or_add_point(sc, state_labels[own[k]], k, cd[k], cc, &Rs);
    covered = (uint8_t *)calloc(obs.n ? (size_t)obs.n : 1, 1);
    if (!covered) { rc = -2; goto out; }
    for (int32_t o = 0; o < n_state; ++o) {
        double lo[3], hi[3];
        or_mesh_box(state_meshes[o], lo, hi);
        for (int32_t p = 0; p < obs.n; ++p)
            if (!covered[p] && or_in_volume(sc, state_labels[o], state_poses + 12 * (size_t)o, lo, hi, &obs, p))
                covered[p] = 1;
    }
    {
        double lo[3], hi[3];
        or_mesh_box(m, lo, hi);
        int err = 0;
#ifdef _OPENMP
        int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(| : err)
#endif
        for (int32_t e = 0; e < n; ++e) {
            const float *P = poses + 12 * (size_t)e;
            valid[e] = 0; jr[e] = 0; jo[e] = 0;
            if (nr) nr[e] = 0;
            if (nq) nq[e] = 0;
            uint16_t *d = (uint16_t *)malloc(N * sizeof(uint16_t));
            uint8_t *c = use_rgb ? (uint8_t *)malloc(3 * N) : NULL;
            or_cloud R;
            if (!d || (use_rgb && !c) || or_cloud_alloc(&R, (size_t)Rs.n + N, use_rgb)) {
                free(d); free(c); err |= 1; continue;
            }
            if (oracle_render(m, P, K, d, NULL, c) != 0) { free(d); free(c); or_cloud_free(&R); err |= 1; continue; }
            int mono = 1;
            for (size_t k = 0; k < N && mono; ++k)
                if (d[k] > 0 && cd[k] > 0 && d[k] < cd[k]) mono = 0;
            if (mono) {
                /* dR \ C, then J_r of each of its points against the observed cloud */
                R.n = 0;
                for (size_t k = 0; k < N; ++k)
                    if (d[k] > 0 && cd[k] == 0) or_add_point(sc, label, k, d[k], c, &R);
                const int32_t n_new = R.n;
                int32_t cr = 0;
                for (int32_t r = 0; r < n_new; ++r) {
                    int32_t nn = -1;
                    int found = or_search(&obs, R.x[r], R.y[r], R.z[r], dq2, dq, use_rgb, &nn);
                    if (!found) cr++;
                    else if (use_rgb && oracle_ciede2000_32(R.lab + 3 * (size_t)r, obs.lab + 3 * (size_t)nn) > sc->tau_c)
                        cr++;
                }
                /* the composed render's points: the state's, then the new object's */
                for (int32_t r = 0; r < Rs.n; ++r) {
                    R.x[R.n] = Rs.x[r]; R.y[R.n] = Rs.y[r]; R.z[R.n] = Rs.z[r]; R.pix[R.n] = Rs.pix[r];
                    if (use_rgb) memcpy(R.lab + 3 * (size_t)R.n, Rs.lab + 3 * (size_t)r, 3 * sizeof(float));
                    R.n++;
                }
                int32_t co = 0, q = 0;
                for (int32_t p = 0; p < obs.n; ++p) {
                    if (covered[p] || !or_in_volume(sc, label, P, lo, hi, &obs, p)) continue;
                    q++;
                    int32_t nn = -1;
                    int found = or_search(&R, obs.x[p], obs.y[p], obs.z[p], dq2, dq, use_rgb, &nn);
                    if (!found) co++;
                    else if (use_rgb && oracle_ciede2000_32(obs.lab + 3 * (size_t)p, R.lab + 3 * (size_t)nn) > sc->tau_c)
                        co++;
                }
                valid[e] = 1; jr[e] = cr; jo[e] = co;
                if (nr) nr[e] = n_new;
                if (nq) nq[e] = q;
            }
            free(d); free(c); or_cloud_free(&R);
        }
        if (err) rc = -2;
    }
out:
    free(cd); free(cc); free(own); free(covered);
    or_cloud_free(&obs); or_cloud_free(&Rs);
    return rc;
}
