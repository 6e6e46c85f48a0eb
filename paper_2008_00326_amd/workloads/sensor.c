/*
 * Sensor simulator for the synthetic RGB-D workloads.
 *
 * Stands in for the photo-realistic renderer that produced the paper's
 * datasets: it casts one ray per pixel centre through a pinhole camera and
 * intersects it with every triangle of every object (Moller-Trumbore, binary64),
 * keeping the nearest hit.  The result is a continuous depth (mm along the
 * optical axis), the barycentric-interpolated vertex colour and the object's
 * label.  Noise and quantisation are added by the Python generator.
 *
 * This is input generation only: it is neither the scoring method nor a
 * model of it, and it shares nothing with the rasterizers that score poses.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
} ss_camera;

static void ss_xform(const double *P, const float *v, double o[3])
{
    double x = v[0], y = v[1], z = v[2];
    o[0] = P[0] * x + P[1] * y + P[2] * z + P[3];
    o[1] = P[4] * x + P[5] * y + P[6] * z + P[7];
    o[2] = P[8] * x + P[9] * y + P[10] * z + P[11];
}

static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

int ss_cast(const ss_camera *cam, int32_t n_obj, const float *const *xyz, const int32_t *n_verts,
            const int32_t *const *tri, const int32_t *n_tris, const uint8_t *const *rgb,
            const double *poses, const int32_t *labels, double *z_out, float *rgb_out,
            int32_t *label_out)
{
    const int W = cam->width, H = cam->height;
    const double near_mm = 1.0;
    for (size_t k = 0; k < (size_t)W * H; ++k) {
        z_out[k] = 0.0;
        label_out[k] = -1;
        rgb_out[3 * k] = rgb_out[3 * k + 1] = rgb_out[3 * k + 2] = 0.0f;
    }
    for (int32_t o = 0; o < n_obj; ++o) {
        const double *P = poses + 12 * (size_t)o;
        double *cv = (double *)malloc(sizeof(double) * 3 * (size_t)n_verts[o]);
        if (!cv) return -2;
        for (int32_t v = 0; v < n_verts[o]; ++v) ss_xform(P, xyz[o] + 3 * (size_t)v, cv + 3 * (size_t)v);
        for (int32_t t = 0; t < n_tris[o]; ++t) {
            const int32_t *ix = tri[o] + 3 * (size_t)t;
            const double *v0 = cv + 3 * (size_t)ix[0], *v1 = cv + 3 * (size_t)ix[1], *v2 = cv + 3 * (size_t)ix[2];
            if (v0[2] <= near_mm || v1[2] <= near_mm || v2[2] <= near_mm) continue;
            double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
            const double *vs[3] = {v0, v1, v2};
            for (int q = 0; q < 3; ++q) {
                double u = cam->fx * vs[q][0] / vs[q][2] + cam->cx;
                double w = cam->fy * vs[q][1] / vs[q][2] + cam->cy;
                if (u < umin) umin = u;
                if (u > umax) umax = u;
                if (w < vmin) vmin = w;
                if (w > vmax) vmax = w;
            }
            int i0 = (int)floor(umin) - 1, i1 = (int)ceil(umax) + 1;
            int j0 = (int)floor(vmin) - 1, j1 = (int)ceil(vmax) + 1;
            if (i0 < 0) i0 = 0;
            if (j0 < 0) j0 = 0;
            if (i1 > W - 1) i1 = W - 1;
            if (j1 > H - 1) j1 = H - 1;
            double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
            double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
            double T[3] = {-v0[0], -v0[1], -v0[2]};
            double Q[3];
            cross3(T, e1, Q);
            for (int j = j0; j <= j1; ++j) {
                for (int i = i0; i <= i1; ++i) {
                    double D[3] = {(i - cam->cx) / cam->fx, (j - cam->cy) / cam->fy, 1.0};
                    double Pv[3];
                    cross3(D, e2, Pv);
                    double det = dot3(e1, Pv);
                    if (fabs(det) < 1e-15) continue;
                    double inv = 1.0 / det;
                    double u = dot3(T, Pv) * inv;
                    if (u < 0.0 || u > 1.0) continue;
                    double w = dot3(D, Q) * inv;
                    if (w < 0.0 || u + w > 1.0) continue;
                    double z = dot3(e2, Q) * inv;
                    if (z <= near_mm) continue;
                    size_t k = (size_t)j * W + i;
                    if (z_out[k] != 0.0 && z >= z_out[k]) continue;
                    z_out[k] = z;
                    label_out[k] = labels[o];
                    if (rgb[o]) {
                        const uint8_t *c0 = rgb[o] + 3 * (size_t)ix[0];
                        const uint8_t *c1 = rgb[o] + 3 * (size_t)ix[1];
                        const uint8_t *c2 = rgb[o] + 3 * (size_t)ix[2];
                        for (int ch = 0; ch < 3; ++ch)
                            rgb_out[3 * k + ch] = (float)((1.0 - u - w) * c0[ch] + u * c1[ch] + w * c2[ch]);
                    }
                }
            }
        }
        free(cv);
    }
    return 0;
}
