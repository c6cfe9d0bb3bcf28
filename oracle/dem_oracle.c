/*
 * dem_oracle.c -- plain FP64 reference DEM timestep (test infrastructure).
 *
 * Written from the Yade DEM documentation (3rd ed., arXiv 2301.00611):
 *   section 2.1.1  collision detection (here: brute force over all pairs),
 *   section 2.1.2  contact stiffness (series springs),
 *   section 2.1.3  kinematic variables (normal, overlap, contact point, shear),
 *   section 2.1.4  contact model (Cundall-Strack, Mohr-Coulomb cap),
 *   section 2.1.5  motion integration (leapfrog, spherical rotation, eq. 2.9),
 *   section 2.1.6  periodic cell (H, velGrad, cellDist),
 *   class reference: ScGeom, Ig2_Wall_Sphere_ScGeom, Ip2_FrictMat_FrictMat_FrictPhys,
 *   FrictPhys, Law2_ScGeom_FrictPhys_CundallStrack, NewtonIntegrator, Cell.
 *
 * Single thread, O(N^2) pair detection, fixed summation order, no FMA
 * contraction (build with -ffp-contract=off).  Clarity over speed: every step
 * is written in the order the documentation gives it.  This file is the
 * oracle for the GPU path and shares no code with it.
 */
#include "dem_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static char g_err[512];

const char* orc_last_error(void) { return g_err; }

static int fail(int code, const char* msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

/* ------------------------------------------------------------------ types */

/* kind 0: FrictMat (density, young, poisson, friction); kind 1: ViscElMat
 * given by contact time and restitution coefficients (tc, en, et), with the
 * class's default young and poisson used only by the P-wave step. */
typedef struct {
    double density, young, poisson, friction;
    int kind;
    double tc, en, et;
} mat_t;

typedef struct {
    int is_wall;
    /* sphere */
    double x[3], v[3], w[3], q[4]; /* q = (qw, qx, qy, qz) */
    double r, m, I;
    unsigned blocked;
    /* boundary (is_wall): prim 0 = infinite axis-aligned plane (utils.wall),
     * 1 = axis-aligned box [lo, hi] (Box), 2 = triangle fv[0..2] (Facet) */
    int prim;
    int axis, sense;
    double wpos;
    double lo[3], hi[3];
    double fv[3][3];
    /* common */
    int mat;
    double F[3], T[3]; /* resultant of the last step's contacts */
} body_t;

typedef struct {
    long lo, hi;  /* key part 1: (min id, max id) */
    int c[3];     /* key part 2: image of #2 */
    long id1, id2;
    int is_wall;
    double fs[3];    /* shear force on #2, carried between steps */
    double nprev[3]; /* normal of the previous step */
    /* geometry found by the detection pass */
    double det_d[3]; /* branch vector from #1 to (the image of) #2 */
    double det_dd;   /* its squared length */
    double det_pen;  /* overlap of a boundary contact */
    double det_n[3]; /* its normal (from the boundary towards the sphere) */
    double det_R1;   /* the boundary's reference radius */
    /* results of the last evaluation */
    double n[3], pen, pt[3], fn[3], kn, ks;
    double fs_out[3];      /* shear force on #2 as reported: fs plus the shear dashpot's force */
    double f2[3];          /* total force on #2 */
    double t1[3], t2[3];   /* torques on #1 and #2 */
} cont_t;

struct orc_scene {
    orc_params p;
    mat_t* mats;
    int nmat, matcap;
    body_t* b;
    long nb, bcap;
    cont_t* c;
    long nc, ccap;
    double H[9], Hprev[9], L[9], Lprev[9], trsf[9];
    long iter;
    double time;
    double e_kin, e_rot, e_el, e_grav, e_damp, e_plast, e_visc;
};

/* ------------------------------------------------------------ small math */

static double dot3(const double a[3], const double b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

static void cross3(const double a[3], const double b[3], double out[3])
{
    double o0 = a[1] * b[2] - a[2] * b[1];
    double o1 = a[2] * b[0] - a[0] * b[2];
    double o2 = a[0] * b[1] - a[1] * b[0];
    out[0] = o0;
    out[1] = o1;
    out[2] = o2;
}

static void matvec(const double M[9], const double v[3], double out[3])
{
    double o[3];
    for (int i = 0; i < 3; ++i)
        o[i] = (M[3 * i + 0] * v[0] + M[3 * i + 1] * v[1]) + M[3 * i + 2] * v[2];
    memcpy(out, o, sizeof o);
}

static void matmul(const double A[9], const double B[9], double out[9])
{
    double o[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            o[3 * i + j] = (A[3 * i + 0] * B[0 + j] + A[3 * i + 1] * B[3 + j]) + A[3 * i + 2] * B[6 + j];
    memcpy(out, o, sizeof o);
}

/* Inverse by the adjugate; H is a non-degenerate cell matrix. */
static int matinv(const double M[9], double out[9])
{
    double a = M[0], b = M[1], c = M[2], d = M[3], e = M[4], f = M[5], g = M[6], h = M[7], i = M[8];
    double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
    double det = a * A + b * B + c * C;
    if (!(fabs(det) > 0.0)) return 0;
    out[0] = A / det;
    out[1] = -(b * i - c * h) / det;
    out[2] = (b * f - c * e) / det;
    out[3] = B / det;
    out[4] = (a * i - c * g) / det;
    out[5] = -(a * f - c * d) / det;
    out[6] = C / det;
    out[7] = -(a * h - b * g) / det;
    out[8] = (a * e - b * d) / det;
    return 1;
}

static int key_cmp(long lo1, long hi1, const int c1[3], long lo2, long hi2, const int c2[3])
{
    if (lo1 != lo2) return lo1 < lo2 ? -1 : 1;
    if (hi1 != hi2) return hi1 < hi2 ? -1 : 1;
    for (int k = 0; k < 3; ++k)
        if (c1[k] != c2[k]) return c1[k] < c2[k] ? -1 : 1;
    return 0;
}

static int cont_cmp(const void* pa, const void* pb)
{
    const cont_t* a = (const cont_t*)pa;
    const cont_t* b = (const cont_t*)pb;
    return key_cmp(a->lo, a->hi, a->c, b->lo, b->hi, b->c);
}

/* Binary search in a key-sorted contact array; NULL if absent. */
static const cont_t* find_contact(const cont_t* arr, long n, long lo, long hi, const int c[3])
{
    long a = 0, z = n;
    while (a < z) {
        long mid = a + (z - a) / 2;
        int r = key_cmp(arr[mid].lo, arr[mid].hi, arr[mid].c, lo, hi, c);
        if (r == 0) return &arr[mid];
        if (r < 0) a = mid + 1;
        else z = mid;
    }
    return NULL;
}

/* ------------------------------------------------------------- lifecycle */

orc_scene* orc_create(const orc_params* p)
{
    if (!p || !(p->dt > 0.0) || p->damping < 0.0 || p->damping >= 1.0) {
        fail(ORC_EINVAL, "orc_create: need dt > 0 and 0 <= damping < 1");
        return NULL;
    }
    orc_scene* s = (orc_scene*)calloc(1, sizeof *s);
    if (!s) return NULL;
    s->p = *p;
    if (p->periodic) {
        double inv[9];
        if (!matinv(p->hsize, inv)) {
            free(s);
            fail(ORC_EINVAL, "orc_create: singular cell matrix");
            return NULL;
        }
        memcpy(s->H, p->hsize, sizeof s->H);
        memcpy(s->L, p->velgrad, sizeof s->L);
    } else {
        for (int k = 0; k < 9; ++k) s->H[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    memcpy(s->Hprev, s->H, sizeof s->H);
    for (int k = 0; k < 9; ++k) s->trsf[k] = (k % 4 == 0) ? 1.0 : 0.0;
    /* Cell.prevVelGrad starts at zero */
    return s;
}

void orc_destroy(orc_scene* s)
{
    if (!s) return;
    free(s->mats);
    free(s->b);
    free(s->c);
    free(s);
}

int orc_add_material(orc_scene* s, double density, double young, double poisson,
                     double friction_angle, int* out_mat)
{
    if (!s) return fail(ORC_EINVAL, "null scene");
    if (!(density > 0.0) || !(young > 0.0) || !(poisson > -1.0 && poisson <= 0.5) ||
        !(friction_angle >= 0.0 && friction_angle < 1.5707963267948966))
        return fail(ORC_EINVAL, "orc_add_material: bad material constants");
    if (s->nmat == s->matcap) {
        int cap = s->matcap ? 2 * s->matcap : 4;
        mat_t* m = (mat_t*)realloc(s->mats, (size_t)cap * sizeof *m);
        if (!m) return fail(ORC_ENOMEM, "out of memory");
        s->mats = m;
        s->matcap = cap;
    }
    memset(&s->mats[s->nmat], 0, sizeof s->mats[s->nmat]);
    s->mats[s->nmat].density = density;
    s->mats[s->nmat].young = young;
    s->mats[s->nmat].poisson = poisson;
    s->mats[s->nmat].friction = friction_angle;
    if (out_mat) *out_mat = s->nmat;
    s->nmat++;
    return ORC_OK;
}

int orc_add_viscel_material(orc_scene* s, double density, double tc, double en, double et,
                            double friction_angle, int* out_mat)
{
    if (!s) return fail(ORC_EINVAL, "null scene");
    if (!(tc > 0.0) || !(en > 0.0 && en <= 1.0) || !(et > 0.0 && et <= 1.0))
        return fail(ORC_EINVAL, "orc_add_viscel_material: tc > 0 and restitution coefficients in (0, 1]");
    int id;
    int rc = orc_add_material(s, density, 1e9, 0.25, friction_angle, &id);
    if (rc) return rc;
    s->mats[id].kind = 1;
    s->mats[id].tc = tc;
    s->mats[id].en = en;
    s->mats[id].et = et;
    if (out_mat) *out_mat = id;
    return ORC_OK;
}

static int grow_bodies(orc_scene* s, long extra)
{
    if (s->nb + extra <= s->bcap) return ORC_OK;
    long cap = s->bcap ? s->bcap : 16;
    while (cap < s->nb + extra) cap *= 2;
    body_t* nb = (body_t*)realloc(s->b, (size_t)cap * sizeof *nb);
    if (!nb) return fail(ORC_ENOMEM, "out of memory");
    s->b = nb;
    s->bcap = cap;
    return ORC_OK;
}

int orc_add_spheres(orc_scene* s, long n, const double* pos3, const double* radius,
                    const double* vel3, const double* angvel3, const int* mat,
                    int default_mat, const unsigned char* blocked, long* out_first_id)
{
    if (!s || n < 0 || (n > 0 && (!pos3 || !radius))) return fail(ORC_EINVAL, "orc_add_spheres: bad arguments");
    for (long i = 0; i < n; ++i) {
        int mi = mat ? mat[i] : default_mat;
        if (mi < 0 || mi >= s->nmat) return fail(ORC_EINVAL, "orc_add_spheres: unknown material");
        if (!(radius[i] > 0.0) || !isfinite(radius[i])) return fail(ORC_EINVAL, "orc_add_spheres: radius must be > 0");
        for (int k = 0; k < 3; ++k)
            if (!isfinite(pos3[3 * i + k])) return fail(ORC_EINVAL, "orc_add_spheres: non-finite position");
    }
    int rc = grow_bodies(s, n);
    if (rc) return rc;
    if (out_first_id) *out_first_id = s->nb;
    for (long i = 0; i < n; ++i) {
        body_t* b = &s->b[s->nb++];
        memset(b, 0, sizeof *b);
        b->is_wall = 0;
        b->mat = mat ? mat[i] : default_mat;
        b->r = radius[i];
        for (int k = 0; k < 3; ++k) {
            b->x[k] = pos3[3 * i + k];
            b->v[k] = vel3 ? vel3[3 * i + k] : 0.0;
            b->w[k] = angvel3 ? angvel3[3 * i + k] : 0.0;
        }
        b->q[0] = 1.0;
        b->blocked = blocked ? (unsigned)(blocked[i] & 63u) : 0u;
        /* Mass and inertia of a sphere from its material density; the
         * documentation's worked example (r = 1, rho = 1000) prints
         * m = 4188.790204786391 and I = 1675.516081914556253, and the
         * expressions below reproduce both digit for digit. */
        double rho = s->mats[b->mat].density;
        double r = b->r;
        b->m = 4.0 / 3.0 * M_PI * r * r * r * rho;
        b->I = 2.0 * b->m * r * r / 5.0;
    }
    return ORC_OK;
}

int orc_add_wall(orc_scene* s, int axis, double position, int sense, int mat, long* out_id)
{
    if (!s || axis < 0 || axis > 2 || sense < -1 || sense > 1 || !isfinite(position))
        return fail(ORC_EINVAL, "orc_add_wall: bad arguments");
    if (mat < 0 || mat >= s->nmat) return fail(ORC_EINVAL, "orc_add_wall: unknown material");
    if (s->p.periodic) return fail(ORC_EINVAL, "orc_add_wall: walls are not supported in a periodic cell");
    int rc = grow_bodies(s, 1);
    if (rc) return rc;
    if (out_id) *out_id = s->nb;
    body_t* b = &s->b[s->nb++];
    memset(b, 0, sizeof *b);
    b->is_wall = 1;
    b->axis = axis;
    b->sense = sense;
    b->wpos = position;
    b->mat = mat;
    b->q[0] = 1.0;
    return ORC_OK;
}

/* utils.PWaveTimeStep / SpherePWaveTimeStep: dt = r / sqrt(E / rho), the
 * minimum over all spheres.  Worked example in the documentation:
 * r = 1e-3, rho = 2400, E = 30e9 gives 2.8284271247461903e-07. */
int orc_pwave_dt(const orc_scene* s, double* out)
{
    if (!s || !out) return fail(ORC_EINVAL, "null argument");
    double best = INFINITY;
    for (long i = 0; i < s->nb; ++i) {
        const body_t* b = &s->b[i];
        if (b->is_wall) continue;
        const mat_t* m = &s->mats[b->mat];
        double dt = b->r / sqrt(m->young / m->density);
        if (dt < best) best = dt;
    }
    *out = best;
    return ORC_OK;
}

long orc_num_bodies(const orc_scene* s) { return s ? s->nb : -1; }
long orc_num_contacts(const orc_scene* s) { return s ? s->nc : -1; }

int orc_get_counters(const orc_scene* s, long* iter, double* time)
{
    if (!s) return fail(ORC_EINVAL, "null scene");
    if (iter) *iter = s->iter;
    if (time) *time = s->time;
    return ORC_OK;
}

/* ------------------------------------------------------- pair detection */

/* Cell vector shift H*c for an integer image c (section 2.1.6: the integer
 * cellDist multiplied by the current cell gives the offset added to #2). */
static void cell_shift(const double H[9], const int c[3], double out[3])
{
    for (int k = 0; k < 3; ++k)
        out[k] = (H[3 * k + 0] * (double)c[0] + H[3 * k + 1] * (double)c[1]) + H[3 * k + 2] * (double)c[2];
}

/* Exact sphere-sphere test.  The pair is real iff |d|^2 < (r1 + r2)^2 with
 * d = (x2 + H c) - x1, evaluated left to right without contraction.  In a
 * periodic cell the 27 images around the nearest one are tried; more than
 * one real image means the spheres span half the cell (section 2.1.6 forbids
 * that).  Returns the number of real images (0 or 1) or -1. */
static int sphere_pair(const orc_scene* s, const body_t* b1, const body_t* b2,
                       const double Hinv[9], int c_out[3], double d_out[3], double* dd_out)
{
    double sr = b1->r + b2->r;
    double s2 = sr * sr;
    if (!s->p.periodic) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = b2->x[k] - b1->x[k];
        double dd = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        if (!(dd < s2)) return 0;
        c_out[0] = c_out[1] = c_out[2] = 0;
        memcpy(d_out, d, sizeof d);
        *dd_out = dd;
        return 1;
    }
    double raw[3], f[3];
    int c0[3];
    for (int k = 0; k < 3; ++k) raw[k] = b2->x[k] - b1->x[k];
    matvec(Hinv, raw, f);
    for (int k = 0; k < 3; ++k) c0[k] = -(int)floor(f[k] + 0.5);
    int found = 0;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int g = -1; g <= 1; ++g) {
                int c[3] = {c0[0] + a, c0[1] + b, c0[2] + g};
                double sh[3], d[3];
                cell_shift(s->H, c, sh);
                for (int k = 0; k < 3; ++k) d[k] = (b2->x[k] + sh[k]) - b1->x[k];
                double dd = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                if (dd < s2) {
                    if (found) return -1;
                    found = 1;
                    memcpy(c_out, c, sizeof c);
                    memcpy(d_out, d, sizeof d);
                    *dd_out = dd;
                }
            }
    return found;
}

static int add_boundary(orc_scene* s, int mat, long* out_id, body_t** out)
{
    if (mat < 0 || mat >= s->nmat) return fail(ORC_EINVAL, "unknown material");
    if (s->p.periodic) return fail(ORC_EINVAL, "boundaries are not supported in a periodic cell");
    int rc = grow_bodies(s, 1);
    if (rc) return rc;
    if (out_id) *out_id = s->nb;
    body_t* b = &s->b[s->nb++];
    memset(b, 0, sizeof *b);
    b->is_wall = 1;
    b->mat = mat;
    b->q[0] = 1.0;
    *out = b;
    return ORC_OK;
}

/* Box: a fixed axis-aligned box with the given centre and half-sizes. */
int orc_add_box(orc_scene* s, const double* center3, const double* half3, int mat, long* out_id)
{
    if (!s || !center3 || !half3) return fail(ORC_EINVAL, "orc_add_box: null argument");
    for (int k = 0; k < 3; ++k)
        if (!isfinite(center3[k]) || !(half3[k] > 0.0) || !isfinite(half3[k]))
            return fail(ORC_EINVAL, "orc_add_box: finite centre and half-sizes > 0");
    body_t* b;
    int rc = add_boundary(s, mat, out_id, &b);
    if (rc) return rc;
    b->prim = 1;
    for (int k = 0; k < 3; ++k) {
        b->lo[k] = center3[k] - half3[k];
        b->hi[k] = center3[k] + half3[k];
    }
    return ORC_OK;
}

/* Facet: a fixed triangle with vertices v0, v1, v2 (not collinear). */
int orc_add_facet(orc_scene* s, const double* v0, const double* v1, const double* v2, int mat, long* out_id)
{
    if (!s || !v0 || !v1 || !v2) return fail(ORC_EINVAL, "orc_add_facet: null argument");
    const double* v[3] = {v0, v1, v2};
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            if (!isfinite(v[i][k])) return fail(ORC_EINVAL, "orc_add_facet: non-finite vertex");
    double e1[3], e2[3], nn[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = v1[k] - v0[k];
        e2[k] = v2[k] - v0[k];
    }
    cross3(e1, e2, nn);
    if (!(dot3(nn, nn) > 0.0)) return fail(ORC_EINVAL, "orc_add_facet: degenerate triangle");
    body_t* b;
    int rc = add_boundary(s, mat, out_id, &b);
    if (rc) return rc;
    b->prim = 2;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) b->fv[i][k] = v[i][k];
    return ORC_OK;
}

/* Wall.sense: -1 / +1 interact on that side only, 0 on both.  With sense 0
 * the normal follows the side the sphere centre is on (side of 0 = +). */
static int wall_sign(const body_t* w, const body_t* sp)
{
    double delta = sp->x[w->axis] - w->wpos;
    if (w->sense != 0) return w->sense;
    return delta >= 0.0 ? 1 : -1;
}

/* Exact wall-sphere test.  The sphere touches the plane iff its centre is
 * closer than r to it, |x[axis] - p| < r; the overlap is then measured from
 * the interacting side, pen = r - sigma*(x[axis] - p), which for a one-sided
 * wall crossed by the sphere exceeds r and pushes it back to that side. */
static int wall_pair(const body_t* w, const body_t* sp, double* pen_out)
{
    double delta = sp->x[w->axis] - w->wpos;
    if (!(fabs(delta) < sp->r)) return 0;
    int sg = wall_sign(w, sp);
    *pen_out = sp->r - (double)sg * delta;
    return 1;
}

/* Closest point of segment [a, b] to x. */
static void closest_on_segment(const double a[3], const double b[3], const double x[3], double out[3])
{
    double ab[3], ax[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ax[k] = x[k] - a[k];
    }
    double t = dot3(ax, ab) / dot3(ab, ab);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    for (int k = 0; k < 3; ++k) out[k] = a[k] + t * ab[k];
}

/* Closest point of the triangle to x: the projection on its plane when it
 * falls inside (same side of all three edges), else the closest of the
 * three edges' closest points. */
static void closest_on_triangle(const double v[3][3], const double x[3], double out[3])
{
    double e1[3], e2[3], nn[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = v[1][k] - v[0][k];
        e2[k] = v[2][k] - v[0][k];
    }
    cross3(e1, e2, nn);
    double len = sqrt(dot3(nn, nn));
    for (int k = 0; k < 3; ++k) nn[k] /= len;
    double h = (x[0] - v[0][0]) * nn[0] + (x[1] - v[0][1]) * nn[1] + (x[2] - v[0][2]) * nn[2];
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = x[k] - h * nn[k];
    int inside = 1;
    for (int i = 0; i < 3; ++i) {
        const double* a = v[i];
        const double* b = v[(i + 1) % 3];
        double ab[3], ap[3], c[3];
        for (int k = 0; k < 3; ++k) {
            ab[k] = b[k] - a[k];
            ap[k] = p[k] - a[k];
        }
        cross3(ab, ap, c);
        if (dot3(c, nn) < 0.0) inside = 0;
    }
    if (inside) {
        memcpy(out, p, sizeof p);
        return;
    }
    double best = INFINITY;
    for (int i = 0; i < 3; ++i) {
        double q[3], d[3];
        closest_on_segment(v[i], v[(i + 1) % 3], x, q);
        for (int k = 0; k < 3; ++k) d[k] = x[k] - q[k];
        double dd = dot3(d, d);
        if (dd < best) {
            best = dd;
            memcpy(out, q, sizeof q);
        }
    }
}

/* Contact of a sphere with a boundary, its normal (from the boundary
 * towards the sphere centre), overlap and the boundary's reference radius:
 *  - plane (Ig2_Wall_Sphere_ScGeom): as wall_pair, reference radius r;
 *  - box (Ig2_Box_Sphere_ScGeom, the box seen as a virtual sphere of the
 *    same radius, reference radius r): centre outside the box: the closest
 *    point p of the box, touching iff |x - p| < r, n = (x - p)/|x - p|,
 *    overlap r - |x - p|; centre inside: pushed out through the nearest face
 *    (first in the order x-, x+, y-, y+, z-, z+ on a tie), overlap r + depth;
 *  - facet (Ig2_Facet_Sphere_ScGeom, two-sided, reference radius 2r): the
 *    closest point p of the triangle, touching iff |x - p| < r, n = (x - p)/
 *    |x - p| (the face normal (v1 - v0) x (v2 - v0) when the centre lies on
 *    the triangle), overlap r - |x - p|. */
static int boundary_pair(const body_t* w, const body_t* sp, double n[3], double* pen, double* R1)
{
    n[0] = n[1] = n[2] = 0.0;
    if (w->prim == 0) {
        if (!wall_pair(w, sp, pen)) return 0;
        n[w->axis] = (double)wall_sign(w, sp);
        *R1 = sp->r;
        return 1;
    }
    if (w->prim == 1) {
        double p[3];
        int inside = 1;
        for (int k = 0; k < 3; ++k) {
            p[k] = sp->x[k] < w->lo[k] ? w->lo[k] : (sp->x[k] > w->hi[k] ? w->hi[k] : sp->x[k]);
            if (sp->x[k] < w->lo[k] || sp->x[k] > w->hi[k]) inside = 0;
        }
        *R1 = sp->r;
        if (!inside) {
            double d[3] = {sp->x[0] - p[0], sp->x[1] - p[1], sp->x[2] - p[2]};
            double dist = sqrt(dot3(d, d));
            if (!(dist < sp->r)) return 0;
            for (int k = 0; k < 3; ++k) n[k] = d[k] / dist;
            *pen = sp->r - dist;
            return 1;
        }
        int ax = 0, sg = -1;
        double depth = INFINITY;
        for (int k = 0; k < 3; ++k) {
            double dl = sp->x[k] - w->lo[k], dh = w->hi[k] - sp->x[k];
            if (dl < depth) {
                depth = dl;
                ax = k;
                sg = -1;
            }
            if (dh < depth) {
                depth = dh;
                ax = k;
                sg = 1;
            }
        }
        n[ax] = (double)sg;
        *pen = sp->r + depth;
        return 1;
    }
    double p[3] = {0.0, 0.0, 0.0};
    closest_on_triangle(w->fv, sp->x, p);
    double d[3] = {sp->x[0] - p[0], sp->x[1] - p[1], sp->x[2] - p[2]};
    double dist = sqrt(dot3(d, d));
    if (!(dist < sp->r)) return 0;
    if (dist > 0.0) {
        for (int k = 0; k < 3; ++k) n[k] = d[k] / dist;
    } else {
        double e1[3], e2[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = w->fv[1][k] - w->fv[0][k];
            e2[k] = w->fv[2][k] - w->fv[0][k];
        }
        cross3(e1, e2, n);
        double len = sqrt(dot3(n, n));
        for (int k = 0; k < 3; ++k) n[k] /= len;
    }
    *pen = sp->r - dist;
    *R1 = 2.0 * sp->r;
    return 1;
}

/* -------------------------------------------------------- contact model */

static const body_t* body(const orc_scene* s, long id) { return &s->b[id]; }

/* The friction angle of a pair is the smaller of the two materials' (both
 * laws). */
static double pair_tanphi(const mat_t* m1, const mat_t* m2)
{
    return tan(m1->friction < m2->friction ? m1->friction : m2->friction);
}

/* Coulomb slider of both laws: a shear force above fmax is brought back to
 * it, adding the slip's plastic work (|Fs_trial| - Fmax)/ks at force Fmax to
 * *e_plast; returns 1 when it slid. */
static int coulomb_cap(double fs[3], double fmax, double ks, double* e_plast)
{
    double fs_norm = sqrt(dot3(fs, fs));
    if (!(fs_norm > fmax)) return 0;
    *e_plast += (fs_norm - fmax) * fmax / ks;
    double ratio = fmax / fs_norm;
    for (int k = 0; k < 3; ++k) fs[k] = fs[k] * ratio;
    return 1;
}

/* Ip2_FrictMat_FrictMat_FrictPhys: k = (E1 D1)(E2 D2) / (E1 D1 + E2 D2) with
 * D = 2*refR; the shear stiffness uses E*nu in place of E; the friction
 * angle is the smaller of the two (section 2.1.2, class reference). */
static void frict_phys(const mat_t* m1, const mat_t* m2, double R1, double R2,
                       double* kn, double* ks, double* tanphi)
{
    double k1 = m1->young * (2.0 * R1);
    double k2 = m2->young * (2.0 * R2);
    *kn = k1 * k2 / (k1 + k2);
    double s1 = (m1->young * m1->poisson) * (2.0 * R1);
    double s2 = (m2->young * m2->poisson) * (2.0 * R2);
    *ks = s1 * s2 / (s1 + s2);
    *tanphi = pair_tanphi(m1, m2);
}

/* Ip2_ViscElMat_ViscElMat_ViscElPhys from contact time and restitution
 * coefficients (Pournin's formulation): the pair takes the means of the two
 * materials' tc, en and et, and m is the reduced mass m1 m2/(m1 + m2) (the
 * other sphere's own mass against a body that cannot move: a boundary or a
 * sphere with all six DOFs blocked); then
 * (getViscoelasticFromSpheresInteraction with that m)
 *   kn = m (pi^2 + ln^2 en)/tc^2,        cn = -2 m ln(en)/tc,
 *   ks = 2/7 m (pi^2 + ln^2 et)/tc^2,    cs = -2/7 m ln(et)/tc,
 * the values for which a two-body collision lasts tc with normal
 * restitution en.  The friction angle is the smaller of the two. */
static void viscel_phys(const mat_t* m1, const mat_t* m2, const body_t* b1, const body_t* b2,
                        double* kn, double* cn, double* ks, double* cs, double* tanphi)
{
    const double pi = 3.14159265358979323846;
    /* a body that cannot move (a boundary, or a sphere with all six DOFs
     * blocked) leaves the other's own mass */
    const int fixed1 = b1->is_wall || b1->blocked == 63u, fixed2 = !b2->is_wall && b2->blocked == 63u;
    double m = b1->m * b2->m / (b1->m + b2->m);
    if (fixed1 && !fixed2) m = b2->m;
    if (fixed2 && !fixed1) m = b1->m;
    double tc = 0.5 * (m1->tc + m2->tc);
    double len = log(0.5 * (m1->en + m2->en));
    double let = log(0.5 * (m1->et + m2->et));
    *kn = m * (pi * pi + len * len) / (tc * tc);
    *cn = -2.0 * m * len / tc;
    *ks = 2.0 / 7.0 * m * (pi * pi + let * let) / (tc * tc);
    *cs = -2.0 / 7.0 * m * let / tc;
    *tanphi = pair_tanphi(m1, m2);
}

/* Evaluate one real contact: ScGeom update (normal, overlap, contact point,
 * shear rotation, relative velocity), then Law2_ScGeom_FrictPhys_CundallStrack.
 * `d` and `dd` are the branch vector from #1 to (the image of) #2 and its
 * squared length, for sphere-sphere contacts; `pen_wall` is the overlap for
 * a wall.  ct->fs / ct->nprev hold the history on entry and are updated.
 * Adds this contact's elastic energy, plastic dissipation and (visco-elastic
 * law) the work of its dashpots over the step to *e_el / *e_plast / *e_visc. */
static void eval_contact(const orc_scene* s, cont_t* ct, const double d[3], double dd,
                         double pen_wall, double* e_el, double* e_plast, double* e_visc)
{
    const double dt = s->p.dt;
    const body_t* b1 = body(s, ct->id1);
    const body_t* b2 = body(s, ct->id2);
    const mat_t* m1 = &s->mats[b1->mat];
    const mat_t* m2 = &s->mats[b2->mat];
    double n[3], pen, R1, R2, pt[3];
    double v1[3] = {0, 0, 0}, w1[3] = {0, 0, 0}, v2[3], w2[3];
    double alpha;

    if (!ct->is_wall) {
        /* ScGeom: l = |x2 - x1|, n = (x2 - x1)/l, overlap = r1 + r2 - l. */
        double l = sqrt(dd);
        for (int k = 0; k < 3; ++k) n[k] = d[k] / l;
        pen = (b1->r + b2->r) - l;
        if (pen < 0.0) pen = 0.0;
        R1 = b1->r;
        R2 = b2->r;
        /* eq. 2.8 with d0 = r1 + r2: the contact point lies in the middle of
         * the overlap zone. */
        for (int k = 0; k < 3; ++k) pt[k] = b1->x[k] + (R1 - 0.5 * pen) * n[k];
        memcpy(v1, b1->v, sizeof v1);
        memcpy(w1, b1->w, sizeof w1);
        /* relative velocity with the factor (r1 + r2)/l that removes
         * granular ratcheting (ScGeom, Ig2_Sphere_Sphere_ScGeom) */
        alpha = (R1 + R2) / l;
    } else {
        /* a boundary (plane, box, facet) is #1; normal, overlap and its
         * reference radius come from boundary_pair at detection */
        memcpy(n, ct->det_n, sizeof n);
        pen = pen_wall;
        R1 = ct->det_R1;
        R2 = b2->r;
        for (int k = 0; k < 3; ++k) pt[k] = b2->x[k] - (b2->r - 0.5 * pen) * n[k];
        alpha = 1.0;
    }
    memcpy(v2, b2->v, sizeof v2);
    memcpy(w2, b2->w, sizeof w2);
    if (s->p.periodic && !ct->is_wall) {
        /* the image of #2 in cell c moves with the cell: (H - H_prev) c / dt */
        double dH[9], sv[3];
        for (int k = 0; k < 9; ++k) dH[k] = s->H[k] - s->Hprev[k];
        cell_shift(dH, ct->c, sv);
        for (int k = 0; k < 3; ++k) v2[k] += sv[k] / dt;
    }

    const int viscel = m1->kind == 1;   /* the scene's materials are all of one kind */
    double kn, ks, tanphi, cn = 0.0, cs = 0.0;
    if (viscel)
        viscel_phys(m1, m2, b1, b2, &kn, &cn, &ks, &cs, &tanphi);
    else
        frict_phys(m1, m2, R1, R2, &kn, &ks, &tanphi);

    /* Shear update, section 2.1.3 "Shear deformation": the previous shear
     * vector is carried by the rotation of the contact plane (n_prev -> n)
     * and by the mean spin about the normal, both increments taken from the
     * previous vector, then the sliding increment -dt * v12_perp is added.
     * Fs = ks * uT, so the same update is applied to the force. */
    double fs_old[3], rot[3], inc1[3], inc2[3], spinv[3];
    memcpy(fs_old, ct->fs, sizeof fs_old);
    cross3(ct->nprev, n, rot);
    cross3(fs_old, rot, inc1);
    double wsum[3] = {w1[0] + w2[0], w1[1] + w2[1], w1[2] + w2[2]};
    double spin = (dt / 2.0) * dot3(n, wsum);
    for (int k = 0; k < 3; ++k) spinv[k] = spin * n[k];
    cross3(fs_old, spinv, inc2);

    /* v12 = alpha (v2 - v1) - (r2 w2 + r1 w1) x n ; shear part only. */
    double v12[3], rw[3], rwxn[3];
    for (int k = 0; k < 3; ++k) rw[k] = R2 * w2[k] + R1 * w1[k]; /* w1 = 0 for a wall */
    cross3(rw, n, rwxn);
    for (int k = 0; k < 3; ++k) v12[k] = alpha * (v2[k] - v1[k]) - rwxn[k];
    double vn = dot3(n, v12);
    double vs[3];
    for (int k = 0; k < 3; ++k) vs[k] = v12[k] - vn * n[k];

    double fs[3];
    for (int k = 0; k < 3; ++k) fs[k] = ((fs_old[k] - inc1[k]) - inc2[k]) - ks * dt * vs[k];

    double fn_mag, fn[3], fsv[3] = {0.0, 0.0, 0.0};
    if (!viscel) {
        /* Law2_ScGeom_FrictPhys_CundallStrack: repulsive normal force kn*pen
         * on #2, shear force capped at |Fn| tan(phi). */
        fn_mag = kn * pen;
        double fmax = fn_mag * tanphi;
        coulomb_cap(fs, fmax, ks, e_plast);
        *e_el += 0.5 * (fn_mag * fn_mag / kn) + 0.5 * (dot3(fs, fs) / ks);
    } else {
        /* Law2_ScGeom_ViscElPhys_Basic: along the normal a spring kn and a
         * dashpot cn in parallel, the dashpot on the overlap's rate of change
         * -(v2 - v1).n (no tension cut-off: the closed forms of kn and cn
         * assume none); tangentially a spring (the shear force carried and
         * incremented as above) and a dashpot cs on the sliding velocity in
         * parallel, in series with a slider: when the spring's force exceeds
         * tan(phi) times the compressive normal force it is brought back to
         * that bound and the shear dashpot carries nothing. */
        double dv[3];
        for (int k = 0; k < 3; ++k) dv[k] = v2[k] - v1[k];
        double un = dot3(n, dv);
        fn_mag = kn * pen - cn * un;
        double fmax = (fn_mag > 0.0 ? fn_mag : 0.0) * tanphi;
        int slide = coulomb_cap(fs, fmax, ks, e_plast);
        if (!slide)
            for (int k = 0; k < 3; ++k) fsv[k] = -cs * vs[k];
        /* dashpot work over the step: cn un^2 dt + cs |vs|^2 dt (sticking) */
        *e_visc += (cn * un * un + (slide ? 0.0 : cs * dot3(vs, vs))) * dt;
        *e_el += 0.5 * (kn * pen * pen) + 0.5 * (dot3(fs, fs) / ks);
    }
    for (int k = 0; k < 3; ++k) fn[k] = fn_mag * n[k];

    /* total force on #2; torques with branch vectors from the radii
     * (Law2_ScGeom_FrictPhys_CundallStrack.sphericalBodies = true):
     * T1 = (r1 n) x (-F), T2 = (-r2 n) x F. */
    double f2[3], br1[3], br2[3], mf[3];
    for (int k = 0; k < 3; ++k) {
        f2[k] = fn[k] + (fs[k] + fsv[k]);
        mf[k] = -f2[k];
        br1[k] = R1 * n[k];
        br2[k] = -R2 * n[k];
    }
    cross3(br1, mf, ct->t1);
    cross3(br2, f2, ct->t2);
    if (ct->is_wall) ct->t1[0] = ct->t1[1] = ct->t1[2] = 0.0;

    memcpy(ct->fs, fs, sizeof fs);
    for (int k = 0; k < 3; ++k) ct->fs_out[k] = fs[k] + fsv[k];
    memcpy(ct->nprev, n, sizeof n);
    memcpy(ct->n, n, sizeof n);
    memcpy(ct->pt, pt, sizeof pt);
    memcpy(ct->fn, fn, sizeof fn);
    memcpy(ct->f2, f2, sizeof f2);
    ct->pen = pen;
    ct->kn = kn;
    ct->ks = ks;
}

/* Build the list of real contacts at the current positions by brute force,
 * in key order, carrying history from `old` (key-sorted).  New contacts start
 * with Fs = 0 and n_prev = n. */
static int detect_all(const orc_scene* s, const cont_t* old, long nold, cont_t** out, long* nout)
{
    double Hinv[9];
    if (s->p.periodic && !matinv(s->H, Hinv)) return fail(ORC_EPERIODIC, "singular cell");
    long cap = 64, n = 0;
    cont_t* arr = (cont_t*)malloc((size_t)cap * sizeof *arr);
    if (!arr) return fail(ORC_ENOMEM, "out of memory");
    for (long i = 0; i < s->nb; ++i) {
        for (long j = i + 1; j < s->nb; ++j) {
            const body_t* bi = &s->b[i];
            const body_t* bj = &s->b[j];
            if (bi->is_wall && bj->is_wall) continue;
            cont_t ct;
            memset(&ct, 0, sizeof ct);
            ct.lo = i;
            ct.hi = j;
            double d[3] = {0, 0, 0}, dd = 0.0, penw = 0.0;
            if (!bi->is_wall && !bj->is_wall) {
                int r = sphere_pair(s, bi, bj, Hinv, ct.c, d, &dd);
                if (r < 0) {
                    free(arr);
                    return fail(ORC_EPERIODIC, "a pair touches through two periodic images: spheres larger than half the cell");
                }
                if (r == 0) continue;
                ct.id1 = i;
                ct.id2 = j;
                for (int k = 0; k < 3; ++k) ct.n[k] = d[k] / sqrt(dd);
            } else {
                const body_t* w = bi->is_wall ? bi : bj;
                const body_t* sp = bi->is_wall ? bj : bi;
                if (!boundary_pair(w, sp, ct.det_n, &penw, &ct.det_R1)) continue;
                ct.is_wall = 1;
                ct.id1 = bi->is_wall ? i : j;
                ct.id2 = bi->is_wall ? j : i;
                memcpy(ct.n, ct.det_n, sizeof ct.n);
            }
            memcpy(ct.det_d, d, sizeof d);
            ct.det_dd = dd;
            ct.det_pen = penw;
            const cont_t* prev = find_contact(old, nold, ct.lo, ct.hi, ct.c);
            if (prev) {
                memcpy(ct.fs, prev->fs, sizeof ct.fs);
                memcpy(ct.nprev, prev->nprev, sizeof ct.nprev);
            } else {
                memcpy(ct.nprev, ct.n, sizeof ct.nprev);
            }
            if (n == cap) {
                cap *= 2;
                cont_t* na = (cont_t*)realloc(arr, (size_t)cap * sizeof *na);
                if (!na) {
                    free(arr);
                    return fail(ORC_ENOMEM, "out of memory");
                }
                arr = na;
            }
            arr[n++] = ct;
        }
    }
    *out = arr;
    *nout = n;
    return ORC_OK;
}

/* One entry of a body's contact list, for the fixed-order sums. */
typedef struct {
    long body, partner;
    int c[3];
    long ci;
    int side; /* 1: the body is #1, 2: the body is #2 */
} entry_t;

static int entry_cmp(const void* pa, const void* pb)
{
    const entry_t* a = (const entry_t*)pa;
    const entry_t* b = (const entry_t*)pb;
    if (a->body != b->body) return a->body < b->body ? -1 : 1;
    if (a->partner != b->partner) return a->partner < b->partner ? -1 : 1;
    for (int k = 0; k < 3; ++k)
        if (a->c[k] != b->c[k]) return a->c[k] < b->c[k] ? -1 : 1;
    return 0;
}

/* Resultant force and torque of every body: contributions are added one by
 * one in ascending partner id (fixed order, so the result does not depend
 * on how contacts are stored).  #2 receives +F, #1 receives -F. */
static int sum_forces(orc_scene* s)
{
    for (long i = 0; i < s->nb; ++i) {
        memset(s->b[i].F, 0, sizeof s->b[i].F);
        memset(s->b[i].T, 0, sizeof s->b[i].T);
    }
    if (s->nc == 0) return ORC_OK;
    entry_t* e = (entry_t*)malloc((size_t)(2 * s->nc) * sizeof *e);
    if (!e) return fail(ORC_ENOMEM, "out of memory");
    for (long k = 0; k < s->nc; ++k) {
        const cont_t* ct = &s->c[k];
        e[2 * k + 0].body = ct->id1;
        e[2 * k + 0].partner = ct->id2;
        e[2 * k + 0].side = 1;
        e[2 * k + 1].body = ct->id2;
        e[2 * k + 1].partner = ct->id1;
        e[2 * k + 1].side = 2;
        for (int h = 0; h < 2; ++h) {
            e[2 * k + h].ci = k;
            memcpy(e[2 * k + h].c, ct->c, sizeof ct->c);
        }
    }
    qsort(e, (size_t)(2 * s->nc), sizeof *e, entry_cmp);
    for (long k = 0; k < 2 * s->nc; ++k) {
        const cont_t* ct = &s->c[e[k].ci];
        body_t* b = &s->b[e[k].body];
        for (int a = 0; a < 3; ++a) {
            if (e[k].side == 2) {
                b->F[a] += ct->f2[a];
                b->T[a] += ct->t2[a];
            } else {
                b->F[a] += -ct->f2[a];
                b->T[a] += ct->t1[a];
            }
        }
    }
    free(e);
    return ORC_OK;
}

/* ---------------------------------------------------------- integration */

static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

/* Quaternion product a*b, (w, x, y, z). */
static void qmul(const double a[4], const double b[4], double out[4])
{
    double o[4];
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    memcpy(out, o, sizeof o);
}

/* Energy increments of one body's Newton update. */
typedef struct {
    double kin, rot, grav, damp;
} newton_energy;

/* NewtonIntegrator for one sphere (section 2.1.5): gravity is a force m*g
 * that is damped like any other (dampGravity = true); Cundall damping
 * eq. 2.9 per component with the on-step velocity estimate v + a dt/2;
 * leapfrog v+ = v- + a dt, x+ = x + v+ dt; spherical rotation
 * w+ = w- + dt T/I, q+ = dq(w+ dt) q.  Blocked components keep their
 * velocity.  Energies use the mid-step values v-, w- (the documentation's
 * two-step energy example fixes this).  F_in/T_in are the contact
 * resultants. */
static void newton_body(const orc_scene* s, body_t* b, const double F_in[3], const double T_in[3],
                        newton_energy* en)
{
    const double dt = s->p.dt;
    const double lam = s->p.damping;
    double f[3], t[3];
    for (int k = 0; k < 3; ++k) {
        f[k] = F_in[k] + b->m * s->p.gravity[k];
        t[k] = T_in[k];
    }
    en->kin = 0.5 * b->m * dot3(b->v, b->v);
    en->rot = 0.5 * b->I * dot3(b->w, b->w);
    en->grav = 0.0;
    en->damp = 0.0;

    double x0[3], v0[3];
    memcpy(x0, b->x, sizeof x0);
    memcpy(v0, b->v, sizeof v0);
    double homo[3] = {0, 0, 0};
    if (s->p.periodic && s->p.homo_deform > 0) {
        /* Cell.homoDeform: dv = (L - L_prev) x  [+ L v- dt when 2] */
        double dL[9], a1[3], a2[3];
        for (int k = 0; k < 9; ++k) dL[k] = s->L[k] - s->Lprev[k];
        matvec(dL, x0, a1);
        matvec(s->L, v0, a2);
        for (int k = 0; k < 3; ++k) homo[k] = a1[k] + (s->p.homo_deform == 2 ? a2[k] * dt : 0.0);
    }
    for (int k = 0; k < 3; ++k) {
        if (b->blocked & (1u << k)) continue;
        en->grav += -b->m * s->p.gravity[k] * v0[k] * dt;
        if (lam > 0.0) {
            double a = f[k] / b->m;
            double df = -lam * sgn(f[k] * (v0[k] + a * dt / 2.0)) * f[k];
            en->damp += -df * v0[k] * dt;
            f[k] += df;
        }
        b->v[k] = v0[k] + f[k] / b->m * dt + homo[k];
    }
    for (int k = 0; k < 3; ++k) b->x[k] = x0[k] + b->v[k] * dt;

    for (int k = 0; k < 3; ++k) {
        if (b->blocked & (8u << k)) continue;
        if (lam > 0.0 && s->p.damp_rot) {
            /* the torque's share of the damping work, on the mid-step spin w-
             * as for the force (the rotational counterpart of nonviscDamp) */
            double a = t[k] / b->I;
            double dtq = -lam * sgn(t[k] * (b->w[k] + a * dt / 2.0)) * t[k];
            en->damp += -dtq * b->w[k] * dt;
            t[k] += dtq;
        }
        b->w[k] = b->w[k] + t[k] / b->I * dt;
    }
    double wn = sqrt(dot3(b->w, b->w));
    if (wn > 0.0) {
        double half = 0.5 * wn * dt;
        double sh = sin(half) / wn;
        double dq[4] = {cos(half), b->w[0] * sh, b->w[1] * sh, b->w[2] * sh};
        double q[4];
        qmul(dq, b->q, q);
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int k = 0; k < 4; ++k) b->q[k] = q[k] / qn;
    }
}

static int step_one(orc_scene* s)
{
    /* ForceResetter + per-step (non-cumulative) energies */
    s->e_kin = s->e_rot = s->e_el = 0.0;

    /* collider + InteractionLoop: detect, then evaluate every real contact */
    cont_t* nc = NULL;
    long nn = 0;
    int rc = detect_all(s, s->c, s->nc, &nc, &nn);
    if (rc) return rc;
    free(s->c);
    s->c = nc;
    s->nc = nn;
    s->ccap = nn;
    double e_el = 0.0, e_plast = 0.0, e_visc = 0.0;
    for (long k = 0; k < s->nc; ++k) {
        cont_t* ct = &s->c[k];
        eval_contact(s, ct, ct->det_d, ct->det_dd, ct->det_pen, &e_el, &e_plast, &e_visc);
    }
    s->e_el = e_el;
    s->e_plast += e_plast;
    s->e_visc += e_visc;

    rc = sum_forces(s);
    if (rc) return rc;

    /* NewtonIntegrator over spheres in id order */
    for (long i = 0; i < s->nb; ++i) {
        body_t* b = &s->b[i];
        if (b->is_wall) continue;
        newton_energy en;
        newton_body(s, b, b->F, b->T, &en);
        s->e_kin += en.kin;
        s->e_rot += en.rot;
        s->e_grav += en.grav;
        s->e_damp += en.damp;
    }

    if (s->p.periodic) {
        /* F+ = (I + L dt) F, same for H (section 2.1.6) */
        double M[9];
        for (int k = 0; k < 9; ++k) M[k] = (k % 4 == 0 ? 1.0 : 0.0) + s->L[k] * s->p.dt;
        memcpy(s->Hprev, s->H, sizeof s->H);
        matmul(M, s->H, s->H);
        matmul(M, s->trsf, s->trsf);
        memcpy(s->Lprev, s->L, sizeof s->L);
    }

    s->time += s->p.dt;
    s->iter += 1;
    for (long i = 0; i < s->nb; ++i) {
        const body_t* b = &s->b[i];
        if (b->is_wall) continue;
        for (int k = 0; k < 3; ++k)
            if (!isfinite(b->x[k]) || !isfinite(b->v[k])) return fail(ORC_ENONFINITE, "non-finite state after step");
    }
    return ORC_OK;
}

/* The contact laws pair materials of one kind (FrictMat with FrictMat,
 * ViscElMat with ViscElMat): a scene that mixes them has no law for some
 * pairs and is refused. */
static int check_material_kinds(const orc_scene* s)
{
    int kind = -1;
    for (long i = 0; i < s->nb; ++i) {
        int k = s->mats[s->b[i].mat].kind;
        if (kind >= 0 && k != kind) return fail(ORC_EINVAL, "bodies of elastic and visco-elastic materials in one scene");
        kind = k;
    }
    return ORC_OK;
}

int orc_step(orc_scene* s, long nsteps)
{
    if (!s || nsteps < 0) return fail(ORC_EINVAL, "orc_step: bad arguments");
    int rc0 = check_material_kinds(s);
    if (rc0) return rc0;
    for (long i = 0; i < nsteps; ++i) {
        int rc = step_one(s);
        if (rc) return rc;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- access */

/* Reported position of a body: a sphere's centre; a plane's coordinate on
 * its axis (0 elsewhere); a box's centre; a facet's centroid. */
static double boundary_position(const body_t* b, int k)
{
    if (!b->is_wall) return b->x[k];
    if (b->prim == 0) return k == b->axis ? b->wpos : 0.0;
    if (b->prim == 1) return 0.5 * (b->lo[k] + b->hi[k]);
    return (b->fv[0][k] + b->fv[1][k] + b->fv[2][k]) / 3.0;
}

int orc_get_state(const orc_scene* s, double* pos3, double* vel3, double* angvel3,
                  double* ori4, double* force3, double* torque3)
{
    if (!s) return fail(ORC_EINVAL, "null scene");
    for (long i = 0; i < s->nb; ++i) {
        const body_t* b = &s->b[i];
        for (int k = 0; k < 3; ++k) {
            if (pos3) pos3[3 * i + k] = boundary_position(b, k);
            if (vel3) vel3[3 * i + k] = b->v[k];
            if (angvel3) angvel3[3 * i + k] = b->w[k];
            if (force3) force3[3 * i + k] = b->F[k];
            if (torque3) torque3[3 * i + k] = b->T[k];
        }
        if (ori4)
            for (int k = 0; k < 4; ++k) ori4[4 * i + k] = b->q[k];
    }
    return ORC_OK;
}

int orc_get_mass(const orc_scene* s, double* mass, double* inertia)
{
    if (!s) return fail(ORC_EINVAL, "null scene");
    for (long i = 0; i < s->nb; ++i) {
        if (mass) mass[i] = s->b[i].m;
        if (inertia) inertia[i] = s->b[i].I;
    }
    return ORC_OK;
}

int orc_set_state(orc_scene* s, const double* pos3, const double* vel3,
                  const double* angvel3, const double* ori4)
{
    if (!s) return fail(ORC_EINVAL, "null scene");
    for (long i = 0; i < s->nb; ++i) {
        body_t* b = &s->b[i];
        if (b->is_wall) continue;
        for (int k = 0; k < 3; ++k) {
            if (pos3) b->x[k] = pos3[3 * i + k];
            if (vel3) b->v[k] = vel3[3 * i + k];
            if (angvel3) b->w[k] = angvel3[3 * i + k];
        }
        if (ori4)
            for (int k = 0; k < 4; ++k) b->q[k] = ori4[4 * i + k];
    }
    return ORC_OK;
}

int orc_get_contacts(const orc_scene* s, long capacity, orc_contact* out, long* out_count)
{
    if (!s || !out_count) return fail(ORC_EINVAL, "null argument");
    *out_count = s->nc;
    if (capacity < s->nc) return fail(ORC_ECAPACITY, "orc_get_contacts: buffer too small");
    for (long k = 0; k < s->nc; ++k) {
        const cont_t* ct = &s->c[k];
        orc_contact* o = &out[k];
        o->id1 = ct->id1;
        o->id2 = ct->id2;
        memcpy(o->cell, ct->c, sizeof o->cell);
        o->is_wall = ct->is_wall;
        memcpy(o->normal, ct->n, sizeof o->normal);
        o->pen = ct->pen;
        memcpy(o->point, ct->pt, sizeof o->point);
        memcpy(o->fn, ct->fn, sizeof o->fn);
        memcpy(o->fs, ct->fs_out, sizeof o->fs);
        o->kn = ct->kn;
        o->ks = ct->ks;
    }
    return ORC_OK;
}

int orc_set_contacts(orc_scene* s, long n, const long* id1, const long* id2,
                     const int* cell3, const double* fs3, const double* nprev3)
{
    if (!s || n < 0 || (n > 0 && (!id1 || !id2 || !fs3 || !nprev3))) return fail(ORC_EINVAL, "orc_set_contacts: bad arguments");
    cont_t* arr = (cont_t*)calloc((size_t)(n > 0 ? n : 1), sizeof *arr);
    if (!arr) return fail(ORC_ENOMEM, "out of memory");
    for (long k = 0; k < n; ++k) {
        if (id1[k] < 0 || id2[k] < 0 || id1[k] >= s->nb || id2[k] >= s->nb || id1[k] == id2[k]) {
            free(arr);
            return fail(ORC_ERANGE, "orc_set_contacts: body id out of range");
        }
        cont_t* ct = &arr[k];
        ct->lo = id1[k] < id2[k] ? id1[k] : id2[k];
        ct->hi = id1[k] < id2[k] ? id2[k] : id1[k];
        for (int a = 0; a < 3; ++a) {
            ct->c[a] = cell3 ? cell3[3 * k + a] : 0;
            ct->fs[a] = fs3[3 * k + a];
            ct->nprev[a] = nprev3[3 * k + a];
        }
    }
    qsort(arr, (size_t)n, sizeof *arr, cont_cmp);
    for (long k = 1; k < n; ++k)
        if (cont_cmp(&arr[k - 1], &arr[k]) == 0) {
            free(arr);
            return fail(ORC_EINVAL, "orc_set_contacts: duplicate key");
        }
    free(s->c);
    s->c = arr;
    s->nc = n;
    s->ccap = n;
    return ORC_OK;
}

int orc_get_energy(const orc_scene* s, double* out8)
{
    if (!s || !out8) return fail(ORC_EINVAL, "null argument");
    out8[0] = s->e_kin;
    out8[1] = s->e_rot;
    out8[2] = s->e_el;
    out8[3] = s->e_grav;
    out8[4] = s->e_damp;
    out8[5] = s->e_plast;
    out8[6] = (((((s->e_kin + s->e_rot) + s->e_el) + s->e_grav) + s->e_damp) + s->e_plast) + s->e_visc;
    out8[7] = s->e_visc;
    return ORC_OK;
}

/* utils.getStress (Love-Weber stress, utility reference of section 5):
 * sigma_ij = (1/V) sum over the real contacts of f_i l_j, f the force on #2,
 * l the branch vector from #2 to #1 (the negated detection vector), so that
 * repulsion gives negative stress.  Wall contacts are left out. */
int orc_get_stress(const orc_scene* s, double volume, double* sigma9)
{
    if (!s || !sigma9) return fail(ORC_EINVAL, "null argument");
    double V = volume;
    if (!(V > 0.0)) {
        if (!s->p.periodic) return fail(ORC_EINVAL, "orc_get_stress: give the volume of an aperiodic scene");
        const double* H = s->H;
        V = fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                 H[2] * (H[3] * H[7] - H[4] * H[6]));
    }
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (long k = 0; k < s->nc; ++k) {
        const cont_t* ct = &s->c[k];
        if (ct->is_wall) continue;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc[3 * i + j] += ct->f2[i] * (-ct->det_d[j]);
    }
    for (int q = 0; q < 9; ++q) sigma9[q] = acc[q] / V;
    return ORC_OK;
}

int orc_get_cell(const orc_scene* s, double* hsize9, double* trsf9)
{
    if (!s) return fail(ORC_EINVAL, "null scene");
    if (hsize9) memcpy(hsize9, s->H, sizeof s->H);
    if (trsf9) memcpy(trsf9, s->trsf, sizeof s->trsf);
    return ORC_OK;
}

/* O.dt = value: the next steps use it. */
int orc_set_dt(orc_scene* s, double dt)
{
    if (!s) return fail(ORC_EINVAL, "null scene");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(ORC_EINVAL, "orc_set_dt: need a finite dt > 0");
    s->p.dt = dt;
    return ORC_OK;
}

/* Cell.velGrad = L between steps (a boundary controller's action): the next
 * step sees the new L and, as Cell.prevVelGrad, the one of the last step. */
int orc_set_velgrad(orc_scene* s, const double* velgrad9)
{
    if (!s || !velgrad9) return fail(ORC_EINVAL, "null argument");
    if (!s->p.periodic) return fail(ORC_EINVAL, "orc_set_velgrad: the scene is not periodic");
    memcpy(s->L, velgrad9, sizeof s->L);
    return ORC_OK;
}

int orc_detect_pairs(const orc_scene* s, long capacity, long* id1, long* id2, int* cell3, long* out_count)
{
    if (!s || !out_count) return fail(ORC_EINVAL, "null argument");
    cont_t* arr = NULL;
    long n = 0;
    int rc = detect_all(s, NULL, 0, &arr, &n);
    if (rc) return rc;
    *out_count = n;
    if (capacity < n) {
        free(arr);
        return fail(ORC_ECAPACITY, "orc_detect_pairs: buffer too small");
    }
    for (long k = 0; k < n; ++k) {
        id1[k] = arr[k].id1;
        id2[k] = arr[k].id2;
        if (cell3)
            for (int a = 0; a < 3; ++a) cell3[3 * k + a] = arr[k].c[a];
    }
    free(arr);
    return ORC_OK;
}

/* Spot mode: the same detection, law, ordered sum and Newton update as a
 * full step, restricted to the contacts of the sampled bodies. */
int orc_spot_step(const orc_scene* s, long k, const long* ids, double* force3,
                  double* torque3, double* pos3, double* vel3, double* angvel3,
                  double* ori4, long* n_contacts, double* fmag_sum)
{
    if (!s || k < 0 || (k > 0 && !ids)) return fail(ORC_EINVAL, "orc_spot_step: bad arguments");
    int rc0 = check_material_kinds(s);
    if (rc0) return rc0;
    double Hinv[9];
    if (s->p.periodic && !matinv(s->H, Hinv)) return fail(ORC_EPERIODIC, "singular cell");
    for (long q = 0; q < k; ++q) {
        long i = ids[q];
        if (i < 0 || i >= s->nb || s->b[i].is_wall) return fail(ORC_ERANGE, "orc_spot_step: not a sphere id");
        const body_t* bi = &s->b[i];
        double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
        double fsum = 0.0;
        long cnt = 0;
        double e_dummy = 0.0, p_dummy = 0.0, v_dummy = 0.0;
        /* partners in ascending id order, as in the full step */
        for (long j = 0; j < s->nb; ++j) {
            if (j == i) continue;
            const body_t* bj = &s->b[j];
            cont_t ct;
            memset(&ct, 0, sizeof ct);
            ct.lo = i < j ? i : j;
            ct.hi = i < j ? j : i;
            double d[3] = {0, 0, 0}, dd = 0.0, penw = 0.0;
            if (!bj->is_wall) {
                const body_t* b1 = i < j ? bi : bj;
                const body_t* b2 = i < j ? bj : bi;
                int r = sphere_pair(s, b1, b2, Hinv, ct.c, d, &dd);
                if (r < 0) return fail(ORC_EPERIODIC, "a pair touches through two periodic images");
                if (r == 0) continue;
                ct.id1 = ct.lo;
                ct.id2 = ct.hi;
                for (int a = 0; a < 3; ++a) ct.n[a] = d[a] / sqrt(dd);
            } else {
                if (!boundary_pair(bj, bi, ct.det_n, &penw, &ct.det_R1)) continue;
                ct.is_wall = 1;
                ct.id1 = j;
                ct.id2 = i;
                memcpy(ct.n, ct.det_n, sizeof ct.n);
            }
            const cont_t* prev = find_contact(s->c, s->nc, ct.lo, ct.hi, ct.c);
            if (prev) {
                memcpy(ct.fs, prev->fs, sizeof ct.fs);
                memcpy(ct.nprev, prev->nprev, sizeof ct.nprev);
            } else {
                memcpy(ct.nprev, ct.n, sizeof ct.nprev);
            }
            eval_contact(s, &ct, d, dd, penw, &e_dummy, &p_dummy, &v_dummy);
            for (int a = 0; a < 3; ++a) {
                if (ct.id2 == i) {
                    F[a] += ct.f2[a];
                    T[a] += ct.t2[a];
                } else {
                    F[a] += -ct.f2[a];
                    T[a] += ct.t1[a];
                }
            }
            fsum += sqrt(dot3(ct.f2, ct.f2));
            cnt++;
        }
        body_t tmp = *bi;
        newton_energy en;
        newton_body(s, &tmp, F, T, &en);
        for (int a = 0; a < 3; ++a) {
            if (force3) force3[3 * q + a] = F[a];
            if (torque3) torque3[3 * q + a] = T[a];
            if (pos3) pos3[3 * q + a] = tmp.x[a];
            if (vel3) vel3[3 * q + a] = tmp.v[a];
            if (angvel3) angvel3[3 * q + a] = tmp.w[a];
        }
        if (ori4)
            for (int a = 0; a < 4; ++a) ori4[4 * q + a] = tmp.q[a];
        if (n_contacts) n_contacts[q] = cnt;
        if (fmag_sum) fmag_sum[q] = fsum;
    }
    return ORC_OK;
}
