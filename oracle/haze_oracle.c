/*
 * haze_oracle.c -- plain, slow FP64 CPU oracle of the splat-and-trace path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * Everything is double precision and written in the order the paper states it:
 *   - density at voxel centres by SPH kernel splatting and the Gladstone-Dale
 *     map n = 1 + K_GD rho                          (Sec. 3.3.1, Eq. 12)
 *   - grad n = K_GD grad rho by finite differences on the grid, then trilinear
 *     sampling of n and grad n along the ray         (Sec. 3.3.1, Eq. 13)
 *   - the explicit direction/position update        (Sec. 3.3.2, Eq. 16)
 *   - curvature and the clamped adaptive step       (Sec. 3.3.3, Eqs. 17-18)
 *   - fixed-step variant                            (Sec. 4.1)
 *   - straight rays outside the volume              (Fig. 1 caption)
 *   - image formed only by bending, via intersecting the refracted ray with
 *     the scene                                     (Sec. 3.3.2, last paragraph)
 *   - scene surfaces (planar parallelograms, or triangle meshes) met anywhere
 *     along the ray: before the volume, on the chord of any step inside it, or
 *     after it; the first one met ends the ray       (Sec. 3.3.2; Secs. 4.1-4.2)
 *     Every chord and straight segment is tested against every surface by
 *     brute force: the acceleration structure of Sec. 4.1 (a conservative
 *     shell around the geometry) only decides which exact tests to skip, so
 *     the oracle has none.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes):
 *   - splat kernel: M4 cubic spline, support 2h, sigma = 1/(pi h^3); plain
 *     (un-normalised) SPH sum  delta_n(c) = K_GD sum_j m_j W(|c - x_j|, h)
 *   - gradient: second-order central differences inside, first-order one-sided
 *     differences on the faces (numpy.gradient with edge_order=1)
 *   - sampling: cell index clamped to [0, R-2], so the outer half-voxel is a
 *     linear extrapolation
 *   - adaptive step uses the second form of Eq. 18:
 *       ds = clamp(n theta / (|P g| + eps), ds_min, ds_max)
 *   - termination: a step never runs past the box; it is shortened to the exit
 *     distance along the current direction, the march stops when that distance
 *     is <= tau or when the new position lies outside the box.
 *
 * Analytic media (constant, linear, n^2 linear, spherical Gaussian) let the
 * same integrator be pinned to closed-form ray paths independently of the grid.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HO_PI 3.14159265358979323846

enum { HO_OK = 0, HO_MAXSTEPS = 1, HO_NOHIT = 2, HO_NONFINITE = 3 };
enum { HO_MEDIUM_GRID = 0, HO_MEDIUM_CONST = 1, HO_MEDIUM_LINEAR = 2, HO_MEDIUM_NSQ_LINEAR = 3,
       HO_MEDIUM_GAUSS = 4 };

typedef struct {
    double lo[3], hi[3];
    int32_t res[3];                 /* Rx, Ry, Rz; arrays are [z][y][x] */
} ho_grid;

/* A refractive medium inside the box [lo, hi] of `grid`.
 *   GRID:        dn, gx, gy, gz sampled trilinearly (Sec. 3.3.1)
 *   CONST:       n = 1 + p[0]
 *   LINEAR:      n = 1 + p[0] + p[1] x + p[2] y + p[3] z
 *   NSQ_LINEAR:  n^2 = p[0] + p[1] x + p[2] y + p[3] z
 *   GAUSS:       n = 1 + p[0] exp(-|x - (p[1],p[2],p[3])|^2 / (2 p[4]^2))      */
typedef struct {
    int32_t kind;
    ho_grid grid;
    const double *dn, *gx, *gy, *gz;
    double p[8];
} ho_medium;

typedef struct {
    double eye[3], fwd[3], up[3];
    double vfov;
    int32_t width, height;
    double plane_p[3], plane_n[3];
} ho_view;

typedef struct {
    int32_t uniform;
    double theta_max, ds_min, ds_max, eps, ds_uniform;
    int64_t max_steps;
    double tau_term;
} ho_step;

/* A scene surface: the parallelogram o + u ea + v eb, 0 <= u, v <= 1, seen
 * from either side. */
typedef struct {
    double o[3], ea[3], eb[3];
} ho_quad;

/* A scene triangle v0 + u e1 + v e2, u, v >= 0, u + v <= 1, seen from either
 * side; `surf` is the surface (mesh part) it belongs to. */
typedef struct {
    double v0[3], e1[3], e2[3];
    int32_t surf;
} ho_tri;

/* The surfaces of one trace: quads (surface k is quad k) and triangles
 * (surface tris[i].surf); a hit reports its surface. */
typedef struct {
    const ho_quad *quads;
    int32_t nq;
    const ho_tri *tris;
    int32_t nt;
} ho_scene;

/* ------------------------------------------------------------------ */
/* small vector helpers                                               */
/* ------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize3(double a[3])
{
    double l = sqrt(dot3(a, a));
    a[0] /= l; a[1] /= l; a[2] /= l;
}
static int finite3(const double a[3]) { return isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]); }

/* ------------------------------------------------------------------ */
/* SPH kernel and splat (Sec. 3.3.1, Eq. 12)                          */
/* ------------------------------------------------------------------ */

/* M4 cubic spline W(r, h) with support 2h and normalisation 1/(pi h^3). */
double ho_kernel(double r, double h)
{
    double q = r / h, w;
    if (q < 1.0)
        w = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    else if (q < 2.0)
        w = 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
    else
        w = 0.0;
    return w / (HO_PI * h * h * h);
}

static double spacing(const ho_grid *g, int a) { return (g->hi[a] - g->lo[a]) / (double)g->res[a]; }
static double centre(const ho_grid *g, int a, int i) { return g->lo[a] + ((double)i + 0.5) * spacing(g, a); }

/* Brute force: every voxel against every particle.  delta_n = K_GD sum_j m_j W. */
void ho_splat_brute(int64_t n, const float *x, const float *y, const float *z, const float *m,
                    const ho_grid *g, double k_gd, double h, double *dn)
{
    const int64_t nx = g->res[0], ny = g->res[1], nz = g->res[2];
    const int64_t nv = nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < nv; ++v) {
        int64_t i = v % nx, j = (v / nx) % ny, k = v / (nx * ny);
        double c[3] = {centre(g, 0, (int)i), centre(g, 1, (int)j), centre(g, 2, (int)k)};
        double rho = 0.0;
        for (int64_t p = 0; p < n; ++p) {
            double dx = c[0] - (double)x[p], dy = c[1] - (double)y[p], dz = c[2] - (double)z[p];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            rho += (double)m[p] * ho_kernel(r, h);
        }
        dn[v] = k_gd * rho;
    }
}

/* Same sum through the oracle's own cell list (cells of edge >= 2h over the
 * particles' bounding box); only particles in the 27 neighbouring cells can be
 * within the support, every other term is exactly zero. */
int ho_splat_cells(int64_t n, const float *x, const float *y, const float *z, const float *m,
                   const ho_grid *g, double k_gd, double h, double *dn)
{
    const int64_t nx = g->res[0], ny = g->res[1], nz = g->res[2];
    const int64_t nv = nx * ny * nz;
    if (n <= 0) {
        for (int64_t v = 0; v < nv; ++v) dn[v] = 0.0;
        return 0;
    }
    double blo[3] = {x[0], y[0], z[0]}, bhi[3] = {x[0], y[0], z[0]};
    for (int64_t p = 1; p < n; ++p) {
        double q[3] = {x[p], y[p], z[p]};
        for (int a = 0; a < 3; ++a) {
            if (q[a] < blo[a]) blo[a] = q[a];
            if (q[a] > bhi[a]) bhi[a] = q[a];
        }
    }
    const double cell = 2.0 * h;
    int64_t cn[3];
    for (int a = 0; a < 3; ++a) {
        cn[a] = (int64_t)floor((bhi[a] - blo[a]) / cell) + 1;
        if (cn[a] < 1) cn[a] = 1;
    }
    const int64_t ncell = cn[0] * cn[1] * cn[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!head || !order || !cid) {
        free(head); free(order); free(cid);
        return -1;
    }
    memset(head, 0, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t p = 0; p < n; ++p) {
        double q[3] = {x[p], y[p], z[p]};
        int64_t ci[3];
        for (int a = 0; a < 3; ++a) {
            ci[a] = (int64_t)floor((q[a] - blo[a]) / cell);
            if (ci[a] < 0) ci[a] = 0;
            if (ci[a] >= cn[a]) ci[a] = cn[a] - 1;
        }
        cid[p] = (ci[2] * cn[1] + ci[1]) * cn[0] + ci[0];
        head[cid[p] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
        if (!fill) {
            free(head); free(order); free(cid);
            return -1;
        }
        memcpy(fill, head, sizeof(int64_t) * (size_t)ncell);
        for (int64_t p = 0; p < n; ++p) order[fill[cid[p]]++] = p;
        free(fill);
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < nv; ++v) {
        int64_t i = v % nx, j = (v / nx) % ny, k = v / (nx * ny);
        double c[3] = {centre(g, 0, (int)i), centre(g, 1, (int)j), centre(g, 2, (int)k)};
        int64_t cc[3];
        for (int a = 0; a < 3; ++a) cc[a] = (int64_t)floor((c[a] - blo[a]) / cell);
        double rho = 0.0;
        for (int64_t dk = -1; dk <= 1; ++dk)
            for (int64_t dj = -1; dj <= 1; ++dj)
                for (int64_t di = -1; di <= 1; ++di) {
                    int64_t q0 = cc[0] + di, q1 = cc[1] + dj, q2 = cc[2] + dk;
                    if (q0 < 0 || q1 < 0 || q2 < 0 || q0 >= cn[0] || q1 >= cn[1] || q2 >= cn[2]) continue;
                    int64_t cell_id = (q2 * cn[1] + q1) * cn[0] + q0;
                    for (int64_t s = head[cell_id]; s < head[cell_id + 1]; ++s) {
                        int64_t p = order[s];
                        double dx = c[0] - (double)x[p], dy = c[1] - (double)y[p], dz = c[2] - (double)z[p];
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        rho += (double)m[p] * ho_kernel(r, h);
                    }
                }
        dn[v] = k_gd * rho;
    }
    free(head); free(order); free(cid);
    return 0;
}

/* ------------------------------------------------------------------ */
/* finite-difference gradient (Sec. 3.3.1, Eq. 13)                    */
/* ------------------------------------------------------------------ */
void ho_gradient(const double *dn, const ho_grid *g, double *gx, double *gy, double *gz)
{
    const int64_t R[3] = {g->res[0], g->res[1], g->res[2]};
    const int64_t stride[3] = {1, R[0], R[0] * R[1]};
    double *out[3] = {gx, gy, gz};
    const int64_t nv = R[0] * R[1] * R[2];
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        int64_t idx[3] = {v % R[0], (v / R[0]) % R[1], v / (R[0] * R[1])};
        for (int a = 0; a < 3; ++a) {
            double d = spacing(g, a);
            int64_t i = idx[a], s = stride[a];
            double val;
            if (i == 0)
                val = (dn[v + s] - dn[v]) / d;
            else if (i == R[a] - 1)
                val = (dn[v] - dn[v - s]) / d;
            else
                val = (dn[v + s] - dn[v - s]) / (2.0 * d);
            out[a][v] = val;
        }
    }
}

/* ------------------------------------------------------------------ */
/* medium sampling: n and grad n at a point                           */
/* ------------------------------------------------------------------ */

/* Trilinear interpolation of a [z][y][x] array at fractional cell coords. */
static double trilinear(const double *f, const int64_t R[3], const int64_t i[3], const double t[3])
{
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
        int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        double w = (bx ? t[0] : 1.0 - t[0]) * (by ? t[1] : 1.0 - t[1]) * (bz ? t[2] : 1.0 - t[2]);
        int64_t v = ((i[2] + bz) * R[1] + (i[1] + by)) * R[0] + (i[0] + bx);
        acc += w * f[v];
    }
    return acc;
}

void ho_sample(const ho_medium *md, const double x[3], double *n_out, double g_out[3])
{
    switch (md->kind) {
    case HO_MEDIUM_GRID: {
        const ho_grid *g = &md->grid;
        int64_t R[3] = {g->res[0], g->res[1], g->res[2]}, i[3];
        double t[3];
        for (int a = 0; a < 3; ++a) {
            double u = (x[a] - g->lo[a]) / spacing(g, a) - 0.5;
            double fl = floor(u);
            if (fl < 0.0) fl = 0.0;
            if (fl > (double)(R[a] - 2)) fl = (double)(R[a] - 2);
            i[a] = (int64_t)fl;
            t[a] = u - fl;
        }
        *n_out = 1.0 + trilinear(md->dn, R, i, t);
        g_out[0] = trilinear(md->gx, R, i, t);
        g_out[1] = trilinear(md->gy, R, i, t);
        g_out[2] = trilinear(md->gz, R, i, t);
        break;
    }
    case HO_MEDIUM_CONST:
        *n_out = 1.0 + md->p[0];
        g_out[0] = g_out[1] = g_out[2] = 0.0;
        break;
    case HO_MEDIUM_LINEAR:
        *n_out = 1.0 + md->p[0] + md->p[1] * x[0] + md->p[2] * x[1] + md->p[3] * x[2];
        g_out[0] = md->p[1]; g_out[1] = md->p[2]; g_out[2] = md->p[3];
        break;
    case HO_MEDIUM_NSQ_LINEAR: {
        double n2 = md->p[0] + md->p[1] * x[0] + md->p[2] * x[1] + md->p[3] * x[2];
        double n = sqrt(n2);
        *n_out = n;
        g_out[0] = md->p[1] / (2.0 * n); g_out[1] = md->p[2] / (2.0 * n); g_out[2] = md->p[3] / (2.0 * n);
        break;
    }
    case HO_MEDIUM_GAUSS: {
        double d[3] = {x[0] - md->p[1], x[1] - md->p[2], x[2] - md->p[3]};
        double s2 = md->p[4] * md->p[4];
        double e = md->p[0] * exp(-dot3(d, d) / (2.0 * s2));
        *n_out = 1.0 + e;
        g_out[0] = -e * d[0] / s2; g_out[1] = -e * d[1] / s2; g_out[2] = -e * d[2] / s2;
        break;
    }
    default:
        *n_out = NAN;
        g_out[0] = g_out[1] = g_out[2] = NAN;
    }
}

/* ------------------------------------------------------------------ */
/* box geometry                                                       */
/* ------------------------------------------------------------------ */

/* Slab test of the line o + t d against [lo, hi]; returns 1 and the entry and
 * exit parameters when the line meets the box. */
static int slab(const double lo[3], const double hi[3], const double o[3], const double d[3],
                double *t_in, double *t_out)
{
    double a = -INFINITY, b = INFINITY;
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) {
            if (o[k] < lo[k] || o[k] > hi[k]) return 0;
            continue;
        }
        double t1 = (lo[k] - o[k]) / d[k], t2 = (hi[k] - o[k]) / d[k];
        if (t1 > t2) { double s = t1; t1 = t2; t2 = s; }
        if (t1 > a) a = t1;
        if (t2 < b) b = t2;
    }
    if (a > b) return 0;
    *t_in = a;
    *t_out = b;
    return 1;
}

/* Distance along d from a point inside the box to the face it leaves through. */
static double exit_distance(const double lo[3], const double hi[3], const double c[3], const double d[3])
{
    double t = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double tk;
        if (d[k] > 0.0)
            tk = (hi[k] - c[k]) / d[k];
        else if (d[k] < 0.0)
            tk = (lo[k] - c[k]) / d[k];
        else
            continue;
        if (tk < t) t = tk;
    }
    return t < 0.0 ? 0.0 : t;
}

static int inside(const double lo[3], const double hi[3], const double c[3])
{
    for (int k = 0; k < 3; ++k)
        if (!(c[k] >= lo[k] && c[k] <= hi[k])) return 0;
    return 1;
}

/* Is the point h, on the plane of q, inside the parallelogram?  Solves
 * h - o = u ea + v eb + s (ea x eb) by Cramer's rule. */
static int in_quad(const ho_quad *q, const double h[3])
{
    double nrm[3], r[3] = {h[0] - q->o[0], h[1] - q->o[1], h[2] - q->o[2]}, c[3];
    cross3(q->ea, q->eb, nrm);
    double det = dot3(nrm, nrm); /* det[ea eb nrm] = (ea x eb) . nrm */
    cross3(r, q->eb, c);
    double u = dot3(c, nrm) / det; /* det[r eb nrm] */
    cross3(q->ea, r, c);
    double v = dot3(c, nrm) / det; /* det[ea r nrm] */
    return u >= 0.0 && u <= 1.0 && v >= 0.0 && v <= 1.0;
}

/* Signed distance-like value (h - o) . (ea x eb) of h from the plane of q. */
static double quad_side(const ho_quad *q, const double h[3])
{
    double nrm[3], r[3] = {h[0] - q->o[0], h[1] - q->o[1], h[2] - q->o[2]};
    cross3(q->ea, q->eb, nrm);
    return dot3(r, nrm);
}

/* Is the point h, on the plane of triangle t, inside it?  The same Cramer
 * solve as in_quad, with the triangle's condition u, v >= 0, u + v <= 1. */
static int in_tri(const ho_tri *t, const double h[3])
{
    double nrm[3], r[3] = {h[0] - t->v0[0], h[1] - t->v0[1], h[2] - t->v0[2]}, c[3];
    cross3(t->e1, t->e2, nrm);
    double det = dot3(nrm, nrm);
    cross3(r, t->e2, c);
    double u = dot3(c, nrm) / det;
    cross3(t->e1, r, c);
    double v = dot3(c, nrm) / det;
    return u >= 0.0 && v >= 0.0 && u + v <= 1.0;
}

/* (h - v0) . (e1 x e2): the side of the triangle's plane h lies on. */
static double tri_side(const ho_tri *t, const double h[3])
{
    double nrm[3], r[3] = {h[0] - t->v0[0], h[1] - t->v0[1], h[2] - t->v0[2]};
    cross3(t->e1, t->e2, nrm);
    return dot3(r, nrm);
}

/* Surface j of a scene (quads first, then triangles): its plane side value
 * at h, whether h (on its plane) lies on it, the plane normal, and the
 * surface id a hit reports. */
static double surf_side(const ho_scene *sc, int32_t j, const double h[3])
{
    return j < sc->nq ? quad_side(&sc->quads[j], h) : tri_side(&sc->tris[j - sc->nq], h);
}
static int surf_inside(const ho_scene *sc, int32_t j, const double h[3])
{
    return j < sc->nq ? in_quad(&sc->quads[j], h) : in_tri(&sc->tris[j - sc->nq], h);
}
static void surf_normal(const ho_scene *sc, int32_t j, double nrm[3])
{
    if (j < sc->nq)
        cross3(sc->quads[j].ea, sc->quads[j].eb, nrm);
    else
        cross3(sc->tris[j - sc->nq].e1, sc->tris[j - sc->nq].e2, nrm);
}
static int surf_id(const ho_scene *sc, int32_t j) { return j < sc->nq ? j : sc->tris[j - sc->nq].surf; }

/* First surface met by the straight ray o + t d with t in [0, t_max]; returns
 * its id (or -1) and the parameter t.  Among equal t the one listed first
 * wins. */
static int cast_scene(const ho_scene *sc, const double o[3], const double d[3], double t_max, double *t_hit)
{
    int best = -1;
    double bt = t_max;
    for (int32_t j = 0; j < sc->nq + sc->nt; ++j) {
        double nrm[3];
        surf_normal(sc, j, nrm);
        double dn = dot3(d, nrm);
        if (dn == 0.0) continue;
        double t = -surf_side(sc, j, o) / dn;
        if (!(t >= 0.0) || t > bt || (t == bt && best >= 0)) continue;
        double h[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        if (!surf_inside(sc, j, h)) continue;
        best = surf_id(sc, j);
        bt = t;
    }
    *t_hit = bt;
    return best;
}

/* First surface crossed by the chord a -> b of one step: the side value
 * changes sign, or is zero at b, after being non-zero at a.  Returns its id
 * (or -1) and the fraction lam in (0, 1] along the chord. */
static int chord_scene(const ho_scene *sc, const double a[3], const double b[3], double *lam_hit)
{
    int best = -1;
    double bl = 2.0;
    for (int32_t j = 0; j < sc->nq + sc->nt; ++j) {
        double sa = surf_side(sc, j, a), sb = surf_side(sc, j, b);
        if (sa == 0.0 || (sa > 0.0 && sb > 0.0) || (sa < 0.0 && sb < 0.0)) continue;
        double lam = sa / (sa - sb);
        if (!(lam < bl)) continue;
        double h[3] = {a[0] + lam * (b[0] - a[0]), a[1] + lam * (b[1] - a[1]), a[2] + lam * (b[2] - a[2])};
        if (!surf_inside(sc, j, h)) continue;
        best = surf_id(sc, j);
        bl = lam;
    }
    *lam_hit = bl;
    return best;
}

/* ------------------------------------------------------------------ */
/* step control (Sec. 3.3.3, Eqs. 17-18) and the march (Eq. 16)       */
/* ------------------------------------------------------------------ */

/* Step length at a sample: fixed, or the clamped curvature-driven rule. */
double ho_step_length(const ho_step *st, double n, const double w[3], const double g[3])
{
    if (st->uniform) return st->ds_uniform;
    double wg = dot3(w, g);
    double pg[3] = {g[0] - wg * w[0], g[1] - wg * w[1], g[2] - wg * w[2]};
    double ds = n * st->theta_max / (sqrt(dot3(pg, pg)) + st->eps);
    if (ds < st->ds_min) ds = st->ds_min;
    if (ds > st->ds_max) ds = st->ds_max;
    return ds;
}

/* Curvature magnitude kappa = |(I - w w^T) g| / n (Eq. 17). */
double ho_curvature(double n, const double w[3], const double g[3])
{
    double wg = dot3(w, g);
    double pg[3] = {g[0] - wg * w[0], g[1] - wg * w[1], g[2] - wg * w[2]};
    return sqrt(dot3(pg, pg)) / n;
}

/* One update of Eq. 16 at (c, w): sample n_k and g_k at c, take the step of
 * Eq. 18 (or the fixed step) shortened to at most te, then
 *   omega_{k+1} = normalize(omega_k + ds/n_k (I - omega_k omega_k^T) g_k)
 *   C_{k+1}     = C_k + ds omega_{k+1}.
 * Updates c and w in place and returns n_k. */
double ho_advance(const ho_medium *md, const ho_step *st, double te, double c[3], double w[3])
{
    double n, g[3];
    ho_sample(md, c, &n, g);
    double ds = ho_step_length(st, n, w, g);
    if (ds > te) ds = te;
    double wg = dot3(w, g);
    double wn[3];
    for (int a = 0; a < 3; ++a) wn[a] = w[a] + (ds / n) * (g[a] - wg * w[a]);
    normalize3(wn);
    for (int a = 0; a < 3; ++a) c[a] += ds * wn[a];
    memcpy(w, wn, sizeof(wn));
    return n;
}

/* March one ray from o along unit d.  The ray is straight until it meets the
 * box; inside, Eq. 16 is applied with the step of Eq. 18 (or the fixed step).
 * Returns the status; x_out / w_out get the last position and direction.
 *
 * With scene surfaces (sc non-NULL): a surface met by the straight ray before
 * the box ends the ray there (x_out = o, no steps); inside the box each step's
 * chord C_k -> C_{k+1} is tested and the first surface crossed ends the ray at
 * the crossing point (x_out = that point, w_out = omega_{k+1}).  *surf_out
 * gets the surface id and hit_out the point, or -1 when none was met on the
 * way (the caller then casts the straight exit ray). */
static int march(const ho_medium *md, const ho_step *st, const ho_scene *sc, const double o[3], const double d[3],
                 double x_out[3], double w_out[3], int64_t *steps_out, double hit_out[3], int *surf_out)
{
    const int nq = sc ? sc->nq + sc->nt : 0;
    const double *lo = md->grid.lo, *hi = md->grid.hi;
    double t_in, t_out;
    *steps_out = 0;
    *surf_out = -1;
    memcpy(w_out, d, sizeof(double) * 3);
    if (!slab(lo, hi, o, d, &t_in, &t_out) || t_out <= 0.0) {
        memcpy(x_out, o, sizeof(double) * 3);
        return HO_OK;
    }
    double s0 = t_in > 0.0 ? t_in : 0.0;
    if (nq > 0) {
        double th;
        int qh = cast_scene(sc, o, d, s0, &th);
        if (qh >= 0) {
            memcpy(x_out, o, sizeof(double) * 3);
            for (int a = 0; a < 3; ++a) hit_out[a] = o[a] + th * d[a];
            *surf_out = qh;
            return HO_OK;
        }
    }
    double c[3] = {o[0] + s0 * d[0], o[1] + s0 * d[1], o[2] + s0 * d[2]};
    double w[3] = {d[0], d[1], d[2]};
    int64_t k = 0;
    int status = HO_OK;
    for (;;) {
        double te = exit_distance(lo, hi, c, w);
        if (te <= st->tau_term) break;
        double cp[3] = {c[0], c[1], c[2]};
        double n = ho_advance(md, st, te, c, w);
        ++k;
        if (!finite3(c) || !finite3(w) || !isfinite(n)) {
            status = HO_NONFINITE;
            break;
        }
        if (nq > 0) {
            double lam;
            int qh = chord_scene(sc, cp, c, &lam);
            if (qh >= 0) {
                for (int a = 0; a < 3; ++a) c[a] = cp[a] + lam * (c[a] - cp[a]);
                memcpy(hit_out, c, sizeof(c));
                *surf_out = qh;
                break;
            }
        }
        if (!inside(lo, hi, c)) break;
        if (k >= st->max_steps) {
            status = HO_MAXSTEPS;
            break;
        }
    }
    memcpy(x_out, c, sizeof(c));
    memcpy(w_out, w, sizeof(w));
    *steps_out = k;
    return status;
}

/* Classical fourth-order Runge-Kutta on (x, omega) with dx/ds = omega and
 * domega/ds = (1/n)(I - omega omega^T) grad n (Eq. 15), omega re-normalised
 * after every step, same box/termination handling as `march`.  Used only to
 * cross-check the converged reference. */
static void rk4_rhs(const ho_medium *md, const double x[3], const double w[3], double dx[3], double dw[3])
{
    double n, g[3];
    ho_sample(md, x, &n, g);
    double wg = dot3(w, g);
    for (int a = 0; a < 3; ++a) {
        dx[a] = w[a];
        dw[a] = (g[a] - wg * w[a]) / n;
    }
}

static int march_rk4(const ho_medium *md, double ds_fixed, int64_t max_steps, double tau,
                     const double o[3], const double d[3], double x_out[3], double w_out[3], int64_t *steps_out)
{
    const double *lo = md->grid.lo, *hi = md->grid.hi;
    double t_in, t_out;
    *steps_out = 0;
    memcpy(w_out, d, sizeof(double) * 3);
    if (!slab(lo, hi, o, d, &t_in, &t_out) || t_out <= 0.0) {
        memcpy(x_out, o, sizeof(double) * 3);
        return HO_OK;
    }
    double s0 = t_in > 0.0 ? t_in : 0.0;
    double x[3] = {o[0] + s0 * d[0], o[1] + s0 * d[1], o[2] + s0 * d[2]};
    double w[3] = {d[0], d[1], d[2]};
    int64_t k = 0;
    int status = HO_OK;
    for (;;) {
        double te = exit_distance(lo, hi, x, w);
        if (te <= tau) break;
        double h = ds_fixed < te ? ds_fixed : te;
        double k1x[3], k1w[3], k2x[3], k2w[3], k3x[3], k3w[3], k4x[3], k4w[3], xt[3], wt[3];
        rk4_rhs(md, x, w, k1x, k1w);
        for (int a = 0; a < 3; ++a) { xt[a] = x[a] + 0.5 * h * k1x[a]; wt[a] = w[a] + 0.5 * h * k1w[a]; }
        rk4_rhs(md, xt, wt, k2x, k2w);
        for (int a = 0; a < 3; ++a) { xt[a] = x[a] + 0.5 * h * k2x[a]; wt[a] = w[a] + 0.5 * h * k2w[a]; }
        rk4_rhs(md, xt, wt, k3x, k3w);
        for (int a = 0; a < 3; ++a) { xt[a] = x[a] + h * k3x[a]; wt[a] = w[a] + h * k3w[a]; }
        rk4_rhs(md, xt, wt, k4x, k4w);
        for (int a = 0; a < 3; ++a) {
            x[a] += h / 6.0 * (k1x[a] + 2.0 * k2x[a] + 2.0 * k3x[a] + k4x[a]);
            w[a] += h / 6.0 * (k1w[a] + 2.0 * k2w[a] + 2.0 * k3w[a] + k4w[a]);
        }
        normalize3(w);
        ++k;
        if (!finite3(x) || !finite3(w)) { status = HO_NONFINITE; break; }
        if (!inside(lo, hi, x)) break;
        if (k >= max_steps) { status = HO_MAXSTEPS; break; }
    }
    memcpy(x_out, x, sizeof(x));
    memcpy(w_out, w, sizeof(w));
    *steps_out = k;
    return status;
}

/* ------------------------------------------------------------------ */
/* cameras, backdrop and displacement                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    double eye[3], f[3], r[3], u[3];
    double fpx;
    int32_t w, h;
} cam_frame;

static void camera_frame(const ho_view *v, cam_frame *cf)
{
    memcpy(cf->eye, v->eye, sizeof(cf->eye));
    memcpy(cf->f, v->fwd, sizeof(cf->f));
    normalize3(cf->f);
    cross3(cf->f, v->up, cf->r);
    normalize3(cf->r);
    cross3(cf->r, cf->f, cf->u);
    cf->fpx = 0.5 * (double)v->height / tan(0.5 * v->vfov);
    cf->w = v->width;
    cf->h = v->height;
}

/* Unit direction through the centre of pixel (p, q); q = 0 is the top row. */
static void pixel_ray(const cam_frame *cf, int64_t p, int64_t q, double d[3])
{
    double sx = (double)p + 0.5 - 0.5 * (double)cf->w;
    double sy = (double)q + 0.5 - 0.5 * (double)cf->h;
    for (int a = 0; a < 3; ++a) d[a] = cf->fpx * cf->f[a] + sx * cf->r[a] - sy * cf->u[a];
    normalize3(d);
}

/* Re-projection of a scene point through the pinhole: displacement =
 * projected point - centre of pixel (p, q). */
static int project_disp(const cam_frame *cf, int64_t p, int64_t q, const double hit[3], double disp[2])
{
    double rel[3] = {hit[0] - cf->eye[0], hit[1] - cf->eye[1], hit[2] - cf->eye[2]};
    double xc = dot3(rel, cf->r), yc = dot3(rel, cf->u), zc = dot3(rel, cf->f);
    if (!(zc > 0.0)) return HO_NOHIT;
    double px = 0.5 * (double)cf->w + cf->fpx * xc / zc;
    double py = 0.5 * (double)cf->h - cf->fpx * yc / zc;
    disp[0] = px - ((double)p + 0.5);
    disp[1] = py - ((double)q + 0.5);
    return HO_OK;
}

/* Parameter t >= 0 at which the straight ray x + t w meets the backdrop plane
 * from its front side (w . N < 0), or -1. */
static double backdrop_t(const ho_view *v, const double x[3], const double w[3])
{
    double denom = dot3(w, v->plane_n);
    if (!(denom < 0.0)) return -1.0;
    double dp[3] = {v->plane_p[0] - x[0], v->plane_p[1] - x[1], v->plane_p[2] - x[2]};
    double t = dot3(dp, v->plane_n) / denom;
    return t >= 0.0 ? t : -1.0;
}

/* Straight segment from the exit point to the backdrop plane, re-projected
 * through the same pinhole. */
static int backdrop_disp(const cam_frame *cf, const ho_view *v, int64_t p, int64_t q, const double x[3],
                         const double w[3], double disp[2])
{
    double t = backdrop_t(v, x, w);
    if (t < 0.0) return HO_NOHIT;
    double hit[3] = {x[0] + t * w[0], x[1] + t * w[1], x[2] + t * w[2]};
    return project_disp(cf, p, q, hit, disp);
}

/* Decode a global ray id (views concatenated, row-major pixels). */
static int decode_ray(const ho_view *views, int32_t nviews, int64_t id, int32_t *vi, int64_t *p, int64_t *q)
{
    int64_t base = 0;
    for (int32_t k = 0; k < nviews; ++k) {
        int64_t cnt = (int64_t)views[k].width * views[k].height;
        if (id < base + cnt) {
            int64_t local = id - base;
            *vi = k;
            *p = local % views[k].width;
            *q = local / views[k].width;
            return 1;
        }
        base += cnt;
    }
    return 0;
}

/* Outputs, caller-owned: disp [n][2], exit_pos [n][3], exit_dir [n][3],
 * steps [n], status [n], surface [n] (may be NULL).  ray_ids may be NULL (then
 * ray i is global id i).
 *
 * The image point of a ray is the first scene surface it meets: a quad met
 * before or inside the volume ends the ray (see march); otherwise the straight
 * exit ray is cast against the quads and the view's backdrop plane and the
 * nearest wins (quads win ties).  surface: 0 backdrop, k + 1 quad k, 255 none. */
static int trace_impl(const ho_medium *md, const ho_view *views, int32_t nviews, const ho_scene *sc,
                      const ho_step *st, const int64_t *ray_ids, int64_t nrays, double *disp, double *exit_pos,
                      double *exit_dir, int64_t *steps, uint8_t *status, uint8_t *surface)
{
    const int nq = sc ? sc->nq + sc->nt : 0;
    cam_frame *cfs = (cam_frame *)malloc(sizeof(cam_frame) * (size_t)(nviews > 0 ? nviews : 1));
    if (!cfs) return -1;
    for (int32_t k = 0; k < nviews; ++k) camera_frame(&views[k], &cfs[k]);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t i = 0; i < nrays; ++i) {
        int64_t id = ray_ids ? ray_ids[i] : i, p, q;
        int32_t vi;
        if (!decode_ray(views, nviews, id, &vi, &p, &q)) {
            bad = 1;
            continue;
        }
        double d[3], x[3], w[3], hit[3], dd[2] = {NAN, NAN};
        int64_t k;
        int surf;
        pixel_ray(&cfs[vi], p, q, d);
        int s = march(md, st, sc, cfs[vi].eye, d, x, w, &k, hit, &surf);
        int sid = 255;
        if (s != HO_NONFINITE) {
            if (surf < 0) {
                double tq, tb = backdrop_t(&views[vi], x, w);
                int qh = nq > 0 ? cast_scene(sc, x, w, INFINITY, &tq) : -1;
                if (qh >= 0 && (tb < 0.0 || tq <= tb)) {
                    surf = qh;
                    for (int a = 0; a < 3; ++a) hit[a] = x[a] + tq * w[a];
                } else if (tb >= 0.0) {
                    surf = -2; /* backdrop */
                    for (int a = 0; a < 3; ++a) hit[a] = x[a] + tb * w[a];
                }
            }
            int b = surf == -1 ? HO_NOHIT : project_disp(&cfs[vi], p, q, hit, dd);
            if (b == HO_NOHIT && s == HO_OK) s = HO_NOHIT;
            if (b == HO_NOHIT)
                dd[0] = dd[1] = NAN;
            else
                sid = surf == -2 ? 0 : surf + 1;
        }
        if (surface) surface[i] = (uint8_t)sid;
        disp[2 * i] = dd[0];
        disp[2 * i + 1] = dd[1];
        for (int a = 0; a < 3; ++a) {
            exit_pos[3 * i + a] = x[a];
            exit_dir[3 * i + a] = w[a];
        }
        steps[i] = k;
        status[i] = (uint8_t)s;
    }
    free(cfs);
    return bad ? -2 : 0;
}

int ho_trace_scene(const ho_medium *md, const ho_view *views, int32_t nviews, const ho_quad *quads, int32_t nq,
                   const ho_step *st, const int64_t *ray_ids, int64_t nrays, double *disp, double *exit_pos,
                   double *exit_dir, int64_t *steps, uint8_t *status, uint8_t *surface)
{
    ho_scene sc = {quads, nq, NULL, 0};
    return trace_impl(md, views, nviews, nq > 0 ? &sc : NULL, st, ray_ids, nrays, disp, exit_pos, exit_dir, steps,
                      status, surface);
}

/* ho_trace_scene with a triangle mesh instead of quads: surface ids are the
 * triangles' `surf` values (a hit on triangle i reports tris[i].surf + 1). */
int ho_trace_mesh(const ho_medium *md, const ho_view *views, int32_t nviews, const ho_tri *tris, int32_t nt,
                  const ho_step *st, const int64_t *ray_ids, int64_t nrays, double *disp, double *exit_pos,
                  double *exit_dir, int64_t *steps, uint8_t *status, uint8_t *surface)
{
    ho_scene sc = {NULL, 0, tris, nt};
    return trace_impl(md, views, nviews, nt > 0 ? &sc : NULL, st, ray_ids, nrays, disp, exit_pos, exit_dir, steps,
                      status, surface);
}

int ho_trace_views(const ho_medium *md, const ho_view *views, int32_t nviews, const ho_step *st,
                   const int64_t *ray_ids, int64_t nrays, double *disp, double *exit_pos, double *exit_dir,
                   int64_t *steps, uint8_t *status)
{
    return trace_impl(md, views, nviews, NULL, st, ray_ids, nrays, disp, exit_pos, exit_dir, steps, status, NULL);
}

/* March explicit rays (origin, unit direction) without a camera. */
int ho_trace_rays(const ho_medium *md, const ho_step *st, const double *origins, const double *dirs, int64_t nrays,
                  double *exit_pos, double *exit_dir, int64_t *steps, uint8_t *status)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nrays; ++i) {
        double x[3], w[3];
        int64_t k;
        double hit[3];
        int surf;
        int s = march(md, st, NULL, origins + 3 * i, dirs + 3 * i, x, w, &k, hit, &surf);
        for (int a = 0; a < 3; ++a) {
            exit_pos[3 * i + a] = x[a];
            exit_dir[3 * i + a] = w[a];
        }
        steps[i] = k;
        status[i] = (uint8_t)s;
    }
    return 0;
}

int ho_trace_rays_rk4(const ho_medium *md, double ds, int64_t max_steps, double tau, const double *origins,
                      const double *dirs, int64_t nrays, double *exit_pos, double *exit_dir, int64_t *steps,
                      uint8_t *status)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nrays; ++i) {
        double x[3], w[3];
        int64_t k;
        int s = march_rk4(md, ds, max_steps, tau, origins + 3 * i, dirs + 3 * i, x, w, &k);
        for (int a = 0; a < 3; ++a) {
            exit_pos[3 * i + a] = x[a];
            exit_dir[3 * i + a] = w[a];
        }
        steps[i] = k;
        status[i] = (uint8_t)s;
    }
    return 0;
}

/* Pixel ray directions (for camera pins). */
int ho_pixel_rays(const ho_view *v, const int64_t *pix, int64_t n, double *dirs)
{
    cam_frame cf;
    camera_frame(v, &cf);
    for (int64_t i = 0; i < n; ++i) pixel_ray(&cf, pix[2 * i], pix[2 * i + 1], dirs + 3 * i);
    return 0;
}

/* Displacement of explicit exit rays seen from pixel (p, q) of view v. */
int ho_backdrop(const ho_view *v, const int64_t *pix, const double *x, const double *w, int64_t n, double *disp,
                uint8_t *status)
{
    cam_frame cf;
    camera_frame(v, &cf);
    for (int64_t i = 0; i < n; ++i) {
        double dd[2] = {NAN, NAN};
        int b = backdrop_disp(&cf, v, pix[2 * i], pix[2 * i + 1], x + 3 * i, w + 3 * i, dd);
        disp[2 * i] = b == HO_OK ? dd[0] : NAN;
        disp[2 * i + 1] = b == HO_OK ? dd[1] : NAN;
        status[i] = (uint8_t)b;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* converged reference: the continuous ODE through the same medium    */
/* ------------------------------------------------------------------ */

/* For each ray: fixed steps ds0, ds0/2, ds0/4, ... until successive levels
 * differ by less than tol_px in displacement and tol_dir in exit direction
 * (or max_levels is reached); the result is the Richardson extrapolation
 * 2 f(ds/2) - f(ds) of the last two levels, valid for a first-order scheme.
 * levels_used[i] records the finest level (0 = ds0); converged[i] = 1 when
 * the tolerance was met. */
int ho_reference_views(const ho_medium *md, const ho_view *views, int32_t nviews, const ho_step *st_template,
                       double ds0, int32_t max_levels, double tol_px, double tol_dir, const int64_t *ray_ids,
                       int64_t nrays, double *disp, double *exit_pos, double *exit_dir, int32_t *levels_used,
                       uint8_t *converged)
{
    if (max_levels < 2) return -3;
    cam_frame *cfs = (cam_frame *)malloc(sizeof(cam_frame) * (size_t)(nviews > 0 ? nviews : 1));
    if (!cfs) return -1;
    for (int32_t k = 0; k < nviews; ++k) camera_frame(&views[k], &cfs[k]);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t i = 0; i < nrays; ++i) {
        int64_t id = ray_ids ? ray_ids[i] : i, p, q;
        int32_t vi;
        if (!decode_ray(views, nviews, id, &vi, &p, &q)) {
            bad = 1;
            continue;
        }
        ho_step st = *st_template;
        st.uniform = 1;
        double d[3];
        pixel_ray(&cfs[vi], p, q, d);
        double prev_x[3] = {0, 0, 0}, prev_w[3] = {0, 0, 0}, prev_d[2] = {0, 0};
        double cur_x[3] = {0, 0, 0}, cur_w[3] = {0, 0, 0}, cur_d[2] = {NAN, NAN};
        int have_prev = 0, ok = 0, lvl;
        double ds = ds0;
        for (lvl = 0; lvl < max_levels; ++lvl, ds *= 0.5) {
            int64_t k;
            st.ds_uniform = ds;
            st.max_steps = INT64_MAX;
            double hit[3];
            int surf;
            march(md, &st, NULL, cfs[vi].eye, d, cur_x, cur_w, &k, hit, &surf);
            cur_d[0] = cur_d[1] = NAN;
            backdrop_disp(&cfs[vi], &views[vi], p, q, cur_x, cur_w, cur_d);
            if (have_prev) {
                double ddx = cur_d[0] - prev_d[0], ddy = cur_d[1] - prev_d[1];
                double dw[3] = {cur_w[0] - prev_w[0], cur_w[1] - prev_w[1], cur_w[2] - prev_w[2]};
                double e_px = sqrt(ddx * ddx + ddy * ddy), e_dir = sqrt(dot3(dw, dw));
                if (!isfinite(e_px)) e_px = 0.0; /* no backdrop hit: judge by direction alone */
                if (e_px < tol_px && e_dir < tol_dir) {
                    ok = 1;
                    break;
                }
            }
            if (lvl == max_levels - 1) break; /* keep the previous level for the extrapolation */
            memcpy(prev_x, cur_x, sizeof(cur_x));
            memcpy(prev_w, cur_w, sizeof(cur_w));
            memcpy(prev_d, cur_d, sizeof(cur_d));
            have_prev = 1;
        }
        if (lvl >= max_levels) lvl = max_levels - 1;
        for (int a = 0; a < 2; ++a) disp[2 * i + a] = 2.0 * cur_d[a] - prev_d[a];
        double wr[3];
        for (int a = 0; a < 3; ++a) {
            exit_pos[3 * i + a] = 2.0 * cur_x[a] - prev_x[a];
            wr[a] = 2.0 * cur_w[a] - prev_w[a];
        }
        normalize3(wr);
        for (int a = 0; a < 3; ++a) exit_dir[3 * i + a] = wr[a];
        levels_used[i] = lvl;
        converged[i] = (uint8_t)ok;
    }
    free(cfs);
    return bad ? -2 : 0;
}

int ho_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing of the oracle itself). */
void ho_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
