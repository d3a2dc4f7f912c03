/*
 * sdm_oracle.c -- plain FP64 CPU oracle of the spectral path tracer.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP library.
 *
 * Structure follows the paper:
 *   Sec. 3.1  inverse ray tracing: a ray per pixel, closest hit, a shadow ray
 *             toward each light, reflected/refracted secondaries, stop after a
 *             fixed number of bounces or below an energy threshold;
 *   eq. (3)   light sum over the directional sun;
 *   eq. (1)   glass optical constants n + ik, Fresnel at the interfaces;
 *   Sec. 6    per-location thickness (per-vertex map);
 *   Sec. 4/5  every pixel and every wavelength is computed on its own; work
 *             items are (pixel tile x spectral band) pulled dynamically.
 * Monte Carlo conventions (random-number mapping, camera, sampling, depth)
 * are readings; each one is stated where it is used.
 */
#include "sdm_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-box with two */
/* 32x32->64 multiplies; the key is bumped by the Weyl constants each round.  */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* Reading: uniform in [0, 1) from the top 24 bits, exact in float and double. */
double orc_u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* Reading: counter = (pixel, sample, (vertex + 1) << 16 | call, job), key =
 * the 64-bit seed; the wavelength is not part of the counter, so all
 * wavelengths of a (pixel, sample) draw the same numbers. */
static void draw4(uint64_t seed, uint32_t job, uint32_t pixel, uint32_t sample, int vertex,
                  uint32_t call, double u[4])
{
    uint32_t ctr[4] = {pixel, sample, ((uint32_t)(vertex + 1) << 16) | call, job};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = orc_u01(x[i]);
}

/* ------------------------------------------------------------------------- */
/* Glass optics                                                               */
/* ------------------------------------------------------------------------- */
/* Fresnel amplitude coefficients air -> n~ = n + ik (eq. (1)); cos of the
 * complex refraction angle from Snell's law on the principal branch. */
void orc_fresnel(double cos_i, double n, double k, double *Rs, double *Rp)
{
    if (cos_i > 1.0) cos_i = 1.0;
    if (cos_i < 0.0) cos_i = 0.0;
    double complex nt = n + I * k;
    double sin2 = 1.0 - cos_i * cos_i;
    double complex ct = csqrt(1.0 - sin2 / (nt * nt));
    double complex rs = (cos_i - nt * ct) / (cos_i + nt * ct);
    double complex rp = (nt * cos_i - ct) / (nt * cos_i + ct);
    *Rs = creal(rs * conj(rs));
    *Rp = creal(rp * conj(rp));
}

/* Reading: the in-glass path length uses the real Snell angle. */
double orc_snell_cos_t(double cos_i, double n)
{
    double s2 = 1.0 - cos_i * cos_i;
    if (s2 < 0.0) s2 = 0.0;
    double st = sqrt(s2) / n;
    double c2 = 1.0 - st * st;
    return c2 > 0.0 ? sqrt(c2) : 0.0;
}

/* One polarisation of a slab with interface reflectance r and one-pass
 * internal transmittance tau: sum of the incoherent bounce series. */
static void slab_pol(double r, double tau, double *R, double *T)
{
    if (r >= 1.0) { *R = 1.0; *T = 0.0; return; }
    double den = 1.0 - r * r * tau * tau;
    *R = r + (1.0 - r) * (1.0 - r) * r * tau * tau / den;
    *T = (1.0 - r) * (1.0 - r) * tau / den;
}

/* Reading: Beer-Lambert absorption alpha = 4 pi k / lambda + alpha_tint, path
 * d / cos(theta_t); the exit face reflects with the entry-face reflectance;
 * the reported slab R, T are the averages of the s and p polarisations. */
void orc_slab(double cos_i, double lambda_nm, double d_mm, double n, double k,
              double alpha_tint, double *R, double *T)
{
    double Rs, Rp;
    orc_fresnel(cos_i, n, k, &Rs, &Rp);
    double ct = orc_snell_cos_t(cos_i, n);
    double alpha = 4.0 * PI * k / (lambda_nm * 1e-6) + alpha_tint;
    double ad = alpha * d_mm;
    double tau = (ad == 0.0) ? 1.0 : (ct > 0.0 ? exp(-ad / ct) : 0.0);
    double Rs_, Ts_, Rp_, Tp_;
    slab_pol(Rs, tau, &Rs_, &Ts_);
    slab_pol(Rp, tau, &Rp_, &Tp_);
    *R = 0.5 * (Rs_ + Rp_);
    *T = 0.5 * (Ts_ + Tp_);
}

void orc_slab_batch(int64_t m, const double *cos_i, const double *lambda_nm, const double *d_mm,
                    const double *n, const double *k, const double *alpha_tint, double *R,
                    double *T)
{
    for (int64_t i = 0; i < m; ++i)
        orc_slab(cos_i[i], lambda_nm[i], d_mm[i], n[i], k[i], alpha_tint[i], R + i, T + i);
}

/* ------------------------------------------------------------------------- */
/* Scene                                                                      */
/* ------------------------------------------------------------------------- */
typedef struct {
    double lo[3], hi[3];
    int32_t left, right; /* children, or -1 for a leaf */
    int32_t first, count;
} onode;

typedef struct {
    int32_t type;
    double thick_mm;
    double *albedo, *n, *k, *tint; /* owned copies [n_tab] */
    double density, rmin_um, rmax_um; /* bubbly glass */
    int32_t pane_id;
    int32_t map;                       /* distribution map index, -1 none */
} omat;

typedef struct {
    int32_t W, H;
    int32_t *material;                 /* owned [W*H] */
    double *thick;                     /* owned [W*H] or NULL */
    double gthick;                     /* largest thickness change per unit of s or t */
} omap;

struct orc_scene {
    int32_t nv, nt, n_mat, n_tab;
    double *pos, *vthick, *ng;
    int32_t *idx, *mat;
    omat *mats;
    double *tab_lambda, *sun_E, *sky_L;
    double sun[3];
    double teps;
    onode *nodes;
    int32_t n_nodes;
    int32_t *order; /* triangle ids in leaf order */
    int32_t depth;
    double *uv;     /* [nv*2] or NULL */
    int32_t n_maps;
    omap *maps;
};

static double *dup_d(const double *p, int64_t n)
{
    if (!p || n <= 0) return NULL;
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(q, p, sizeof(double) * (size_t)n);
    return q;
}

static void sub3(const double *a, const double *b, double *r) { for (int i = 0; i < 3; ++i) r[i] = a[i] - b[i]; }
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize3(double *a)
{
    double l = sqrt(dot3(a, a));
    if (l > 0) { a[0] /= l; a[1] /= l; a[2] /= l; }
}

/* Median-split BVH (leaves of at most 4 triangles).  Any acceleration
 * structure gives the same closest hit under the tie rule below; this one is
 * kept simple and is checked against brute force. */
typedef struct { double key; int32_t id; } keyed;
static int cmp_keyed(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id < y->id) ? -1 : (x->id > y->id);
}

static int32_t bvh_build(orc_scene *s, int32_t first, int32_t count, double pad, int depth)
{
    int32_t me = s->n_nodes++;
    onode *nd = &s->nodes[me];
    for (int a = 0; a < 3; ++a) { nd->lo[a] = INFINITY; nd->hi[a] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = first; i < first + count; ++i) {
        int32_t t = s->order[i];
        for (int c = 0; c < 3; ++c) {
            const double *p = s->pos + 3 * s->idx[3 * t + c];
            for (int a = 0; a < 3; ++a) {
                if (p[a] < nd->lo[a]) nd->lo[a] = p[a];
                if (p[a] > nd->hi[a]) nd->hi[a] = p[a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            double cen = (s->pos[3 * s->idx[3 * t] + a] + s->pos[3 * s->idx[3 * t + 1] + a] +
                          s->pos[3 * s->idx[3 * t + 2] + a]) / 3.0;
            if (cen < clo[a]) clo[a] = cen;
            if (cen > chi[a]) chi[a] = cen;
        }
    }
    for (int a = 0; a < 3; ++a) { nd->lo[a] -= pad; nd->hi[a] += pad; }
    if (depth + 1 > s->depth) s->depth = depth + 1;
    if (count <= 4) {
        nd->left = nd->right = -1;
        nd->first = first;
        nd->count = count;
        return me;
    }
    int axis = 0;
    for (int a = 1; a < 3; ++a) if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    keyed *tmp = (keyed *)malloc(sizeof(keyed) * (size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        int32_t t = s->order[first + i];
        tmp[i].key = s->pos[3 * s->idx[3 * t] + axis] + s->pos[3 * s->idx[3 * t + 1] + axis] +
                     s->pos[3 * s->idx[3 * t + 2] + axis];
        tmp[i].id = t;
    }
    qsort(tmp, (size_t)count, sizeof(keyed), cmp_keyed);
    for (int32_t i = 0; i < count; ++i) s->order[first + i] = tmp[i].id;
    free(tmp);
    int32_t half = count / 2;
    nd->first = nd->count = 0;
    int32_t l = bvh_build(s, first, half, pad, depth + 1);
    int32_t r = bvh_build(s, first + half, count - half, pad, depth + 1);
    s->nodes[me].left = l;
    s->nodes[me].right = r;
    return me;
}

orc_scene *orc_scene_create(const orc_scene_desc *d)
{
    if (!d || d->nv < 0 || d->nt < 0 || d->n_tab < 1 || !d->tab_lambda_nm || !d->sun_E || !d->sky_L)
        return NULL;
    if (d->nt > 0 && (!d->pos || !d->idx || !d->mat || !d->mats || d->n_mat < 1)) return NULL;
    for (int32_t t = 0; t < d->nt; ++t) {
        for (int c = 0; c < 3; ++c)
            if (d->idx[3 * t + c] < 0 || d->idx[3 * t + c] >= d->nv) return NULL;
        if (d->mat[t] < 0 || d->mat[t] >= d->n_mat) return NULL;
    }
    for (int32_t m = 0; m < d->n_mat; ++m) {
        const orc_material *mm = &d->mats[m];
        if (mm->type == ORC_LAMBERT && !mm->albedo) return NULL;
        if (mm->type != ORC_LAMBERT && (!mm->n || !mm->k)) return NULL;
        if (mm->dist_map != 0 && (mm->type != ORC_GLASS || mm->dist_map < 0 || mm->dist_map > d->n_maps || !d->uv))
            return NULL;
    }
    if (d->n_maps < 0 || (d->n_maps > 0 && !d->maps)) return NULL;
    for (int32_t q = 0; q < d->n_maps; ++q) {
        const orc_dist_map *dm = &d->maps[q];
        if (dm->W < 1 || dm->H < 1 || !dm->material) return NULL;
        for (int64_t x = 0; x < (int64_t)dm->W * dm->H; ++x) {
            int32_t tm = dm->material[x];
            if (tm < 0 || tm >= d->n_mat || d->mats[tm].type != ORC_GLASS || d->mats[tm].dist_map != 0) return NULL;
            if (dm->thick_mm && !(dm->thick_mm[x] > 0.0)) return NULL;
        }
    }
    orc_scene *s = (orc_scene *)calloc(1, sizeof(orc_scene));
    s->nv = d->nv; s->nt = d->nt; s->n_mat = d->n_mat; s->n_tab = d->n_tab;
    s->pos = dup_d(d->pos, 3 * (int64_t)d->nv);
    s->vthick = dup_d(d->vthick_mm, d->nv);
    s->idx = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(d->nt + 1));
    s->mat = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d->nt + 1));
    if (d->nt) {
        memcpy(s->idx, d->idx, sizeof(int32_t) * 3 * (size_t)d->nt);
        memcpy(s->mat, d->mat, sizeof(int32_t) * (size_t)d->nt);
    }
    s->mats = (omat *)calloc((size_t)(d->n_mat + 1), sizeof(omat));
    for (int32_t m = 0; m < d->n_mat; ++m) {
        const orc_material *mm = &d->mats[m];
        s->mats[m].type = mm->type;
        s->mats[m].thick_mm = mm->thick_mm;
        s->mats[m].albedo = dup_d(mm->albedo, d->n_tab);
        s->mats[m].n = dup_d(mm->n, d->n_tab);
        s->mats[m].k = dup_d(mm->k, d->n_tab);
        s->mats[m].tint = dup_d(mm->alpha_tint, d->n_tab);
        s->mats[m].density = mm->bubble_density;
        s->mats[m].rmin_um = mm->bubble_rmin_um;
        s->mats[m].rmax_um = mm->bubble_rmax_um;
        s->mats[m].pane_id = mm->pane_id;
        s->mats[m].map = mm->dist_map - 1;
    }
    s->uv = dup_d(d->uv, 2 * (int64_t)d->nv);
    s->n_maps = d->n_maps;
    s->maps = (omap *)calloc((size_t)(d->n_maps + 1), sizeof(omap));
    for (int32_t q = 0; q < d->n_maps; ++q) {
        const orc_dist_map *dm = &d->maps[q];
        omap *M = &s->maps[q];
        size_t n = (size_t)dm->W * dm->H;
        M->W = dm->W;
        M->H = dm->H;
        M->material = (int32_t *)malloc(sizeof(int32_t) * n);
        memcpy(M->material, dm->material, sizeof(int32_t) * n);
        M->thick = dup_d(dm->thick_mm, (int64_t)n);
        /* the bilinear surface's slope is at most the largest difference of
         * neighbouring texels times texels per unit */
        M->gthick = 0.0;
        if (M->thick)
            for (int32_t y = 0; y < M->H; ++y)
                for (int32_t x = 0; x < M->W; ++x) {
                    double t0 = M->thick[y * M->W + x];
                    if (x + 1 < M->W) M->gthick = fmax(M->gthick, fabs(M->thick[y * M->W + x + 1] - t0) * M->W);
                    if (y + 1 < M->H) M->gthick = fmax(M->gthick, fabs(M->thick[(y + 1) * M->W + x] - t0) * M->H);
                }
    }
    s->tab_lambda = dup_d(d->tab_lambda_nm, d->n_tab);
    s->sun_E = dup_d(d->sun_E, d->n_tab);
    s->sky_L = dup_d(d->sky_L, d->n_tab);
    for (int a = 0; a < 3; ++a) s->sun[a] = d->sun_dir[a];
    /* geometric normals and the self-intersection epsilon */
    s->ng = (double *)malloc(sizeof(double) * 3 * (size_t)(d->nt + 1));
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t t = 0; t < d->nt; ++t) {
        const double *p0 = s->pos + 3 * s->idx[3 * t], *p1 = s->pos + 3 * s->idx[3 * t + 1],
                     *p2 = s->pos + 3 * s->idx[3 * t + 2];
        double e1[3], e2[3];
        sub3(p1, p0, e1);
        sub3(p2, p0, e2);
        cross3(e1, e2, s->ng + 3 * t);
        normalize3(s->ng + 3 * t);
    }
    for (int32_t v = 0; v < d->nv; ++v)
        for (int a = 0; a < 3; ++a) {
            if (s->pos[3 * v + a] < lo[a]) lo[a] = s->pos[3 * v + a];
            if (s->pos[3 * v + a] > hi[a]) hi[a] = s->pos[3 * v + a];
        }
    double diag = 0.0;
    if (d->nv > 0) {
        double e[3];
        sub3(hi, lo, e);
        diag = sqrt(dot3(e, e));
    }
    /* Reading: hits are accepted for t > 1e-6 x scene diagonal. */
    s->teps = 1e-6 * diag;
    s->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(d->nt + 1));
    for (int32_t t = 0; t < d->nt; ++t) s->order[t] = t;
    s->nodes = (onode *)calloc((size_t)(2 * d->nt + 2), sizeof(onode));
    s->n_nodes = 0;
    if (d->nt > 0) bvh_build(s, 0, d->nt, 1e-9 * (diag + 1.0), 0);
    return s;
}

void orc_scene_destroy(orc_scene *s)
{
    if (!s) return;
    for (int32_t m = 0; m < s->n_mat; ++m) {
        free(s->mats[m].albedo); free(s->mats[m].n); free(s->mats[m].k); free(s->mats[m].tint);
    }
    free(s->mats); free(s->pos); free(s->vthick); free(s->ng); free(s->idx); free(s->mat);
    free(s->tab_lambda); free(s->sun_E); free(s->sky_L); free(s->nodes); free(s->order);
    for (int32_t q = 0; q < s->n_maps; ++q) { free(s->maps[q].material); free(s->maps[q].thick); }
    free(s->maps); free(s->uv);
    free(s);
}

double orc_scene_teps(const orc_scene *s) { return s->teps; }
int32_t orc_bvh_depth(const orc_scene *s) { return s->depth; }

/* ------------------------------------------------------------------------- */
/* Intersection                                                               */
/* ------------------------------------------------------------------------- */
/* Moeller-Trumbore (1997): two-sided, edges inclusive (u, v >= 0, u + v <= 1). */
static int tri_hit(const orc_scene *s, int32_t t, const double *o, const double *d, double *tt,
                   double *uu, double *vv)
{
    const double *p0 = s->pos + 3 * s->idx[3 * t], *p1 = s->pos + 3 * s->idx[3 * t + 1],
                 *p2 = s->pos + 3 * s->idx[3 * t + 2];
    double e1[3], e2[3], pv[3], sv[3], qv[3];
    sub3(p1, p0, e1);
    sub3(p2, p0, e2);
    cross3(d, e2, pv);
    double det = dot3(e1, pv);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    sub3(o, p0, sv);
    double u = dot3(sv, pv) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    cross3(sv, e1, qv);
    double v = dot3(d, qv) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    *tt = dot3(e2, qv) * inv;
    *uu = u;
    *vv = v;
    return 1;
}

typedef struct { double t, u, v; int32_t tri; } ohit;

/* Reading: the closest accepted hit wins; an exact tie in t goes to the
 * smaller triangle index, which makes the result independent of the
 * acceleration structure. */
static void consider(const orc_scene *s, int32_t t, const double *o, const double *d, int32_t skip,
                     ohit *h)
{
    if (t == skip) return;
    double tt, u, v;
    if (!tri_hit(s, t, o, d, &tt, &u, &v)) return;
    if (!(tt > s->teps)) return;
    if (tt < h->t || (tt == h->t && t < h->tri)) { h->t = tt; h->u = u; h->v = v; h->tri = t; }
}

static int box_overlap(const onode *n, const double *o, const double *d, double tlo, double thi)
{
    double a = -INFINITY, b = INFINITY;
    for (int i = 0; i < 3; ++i) {
        if (d[i] == 0.0) {
            if (o[i] < n->lo[i] || o[i] > n->hi[i]) return 0;
            continue;
        }
        double t1 = (n->lo[i] - o[i]) / d[i], t2 = (n->hi[i] - o[i]) / d[i];
        double mn = t1 < t2 ? t1 : t2, mx = t1 < t2 ? t2 : t1;
        if (mn > a) a = mn;
        if (mx < b) b = mx;
    }
    return a <= b && b >= tlo && a <= thi;
}

static ohit closest(const orc_scene *s, int use_bvh, const double *o, const double *d, int32_t skip)
{
    ohit h = {INFINITY, 0, 0, -1};
    if (s->nt == 0) return h;
    if (!use_bvh) {
        for (int32_t t = 0; t < s->nt; ++t) consider(s, t, o, d, skip, &h);
        return h;
    }
    int32_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const onode *n = &s->nodes[stack[--sp]];
        if (!box_overlap(n, o, d, s->teps, h.t)) continue;
        if (n->left < 0) {
            for (int32_t i = n->first; i < n->first + n->count; ++i) consider(s, s->order[i], o, d, skip, &h);
        } else {
            stack[sp++] = n->left;
            stack[sp++] = n->right;
        }
    }
    return h;
}

static double interp_tab(const orc_scene *s, const double *ys, double x);

/* Glass thickness at barycentric (u, v): the per-vertex distribution map. */
/* Magnitude of the gradient of the interpolated thickness across triangle
 * t (mm per metre; 0 without a thickness map).  With e1 = p1 - p0, e2 =
 * p2 - p0 and N = e1 x e2, the barycentric gradients are (e2 x N) / |N|^2
 * and (N x e1) / |N|^2. */
static double thickness_grad(const orc_scene *s, int32_t t)
{
    if (!s->vthick) return 0.0;
    const double *p0 = s->pos + 3 * s->idx[3 * t], *p1 = s->pos + 3 * s->idx[3 * t + 1],
                 *p2 = s->pos + 3 * s->idx[3 * t + 2];
    double e1[3], e2[3], N[3], gu[3], gv[3];
    sub3(p1, p0, e1);
    sub3(p2, p0, e2);
    cross3(e1, e2, N);
    double nn = dot3(N, N);
    if (!(nn > 0.0)) return 0.0;
    cross3(e2, N, gu);
    cross3(N, e1, gv);
    double d0 = s->vthick[s->idx[3 * t]], d1 = s->vthick[s->idx[3 * t + 1]], d2 = s->vthick[s->idx[3 * t + 2]];
    double g[3];
    for (int a = 0; a < 3; ++a) g[a] = ((d1 - d0) * gu[a] + (d2 - d0) * gv[a]) / nn;
    return sqrt(dot3(g, g));
}

/* Hit error of the single-precision bound (see orc_render_params): a hit
 * reached from an origin with error bound e over a distance dist at incidence
 * cosine c, landing at x. */
static double hit_error(const orc_render_params *p, double e, double dist, double c, const double *x)
{
    double ax = fmax(fmax(fabs(x[0]), fabs(x[1])), fabs(x[2]));
    return (e + p->prec_eps * dist) / fmax(c, 1e-300) + p->prec_eps * ax;
}

/* Relative error bound of a glass factor at incidence cosine c with a hit
 * error h on triangle t (see orc_render_params). */
static double glass_sensitivity(const orc_render_params *p, const orc_scene *s, int32_t t, double h, double c,
                                double n, double alpha)
{
    if (!(c > 0.0)) return INFINITY;
    double st = sqrt(fmax(0.0, 1.0 - c * c)) / n, ct = sqrt(fmax(1e-300, 1.0 - st * st));
    return p->prec_ceps / c + alpha * thickness_grad(s, t) * h / ct;
}

static void tex_at(const orc_scene *s, int32_t t, double u, double v, double st[2]);

/* As glass_sensitivity, for the pane of triangle t hit at barycentric (u, v)
 * with hit error h, whose optical constants or thickness may come from a
 * distribution map.  The texture coordinates move by the hit error through
 * the barycentric gradients, plus a few roundings of their interpolation; a
 * hit whose coordinates may cross a texel edge may take another texel's
 * material, and the bound then covers any value (1e30); a thickness table
 * moves by its slope times that error. */
static double pane_sensitivity(const orc_render_params *p, const orc_scene *s, int32_t t, double u, double v,
                               double h, double c, double n, double alpha)
{
    int32_t mp = s->mats[s->mat[t]].map;
    if (mp < 0) return glass_sensitivity(p, s, t, h, c, n, alpha);
    if (!(c > 0.0)) return 1e30;
    const omap *M = &s->maps[mp];
    const double *p0 = s->pos + 3 * s->idx[3 * t], *p1 = s->pos + 3 * s->idx[3 * t + 1],
                 *p2 = s->pos + 3 * s->idx[3 * t + 2];
    double e1[3], e2[3], N[3], gu[3], gv[3];
    sub3(p1, p0, e1);
    sub3(p2, p0, e2);
    cross3(e1, e2, N);
    double nn = dot3(N, N);
    if (!(nn > 0.0)) return 1e30;
    cross3(e2, N, gu);
    cross3(N, e1, gv);
    const double *q0 = s->uv + 2 * s->idx[3 * t], *q1 = s->uv + 2 * s->idx[3 * t + 1],
                 *q2 = s->uv + 2 * s->idx[3 * t + 2];
    double st[2], es[2];
    tex_at(s, t, u, v, st);
    const double ulp = 0.5 * p->prec_eps;
    for (int a = 0; a < 2; ++a) {
        double g[3];
        for (int k = 0; k < 3; ++k) g[k] = ((q1[a] - q0[a]) * gu[k] + (q2[a] - q0[a]) * gv[k]) / nn;
        es[a] = sqrt(dot3(g, g)) * h +
                8.0 * ulp * (fabs(q0[a]) + fabs(q1[a]) + fabs(q2[a]) + fabs(st[a]) + 1.0);
    }
    const int32_t dims[2] = {M->W, M->H};
    for (int a = 0; a < 2; ++a) {
        double x = st[a] * dims[a], ke = nearbyint(x);
        if (ke >= 1.0 && ke <= (double)(dims[a] - 1) && fabs(x - ke) <= es[a] * dims[a] * 1.01 + 8.0 * ulp * fabs(x))
            return 1e30;
    }
    int32_t me;
    double d;
    orc_pane_at(s, t, u, v, &me, &d);
    double dd = M->thick ? M->gthick * fmax(es[0], es[1]) : thickness_grad(s, t) * h;
    dd += 8.0 * ulp * d;
    double sn = sqrt(fmax(0.0, 1.0 - c * c)) / n, ct = sqrt(fmax(1e-300, 1.0 - sn * sn));
    return p->prec_ceps / c + alpha * dd / ct;
}

static double thickness_at(const orc_scene *s, int32_t t, double u, double v)
{
    const omat *m = &s->mats[s->mat[t]];
    if (!s->vthick) return m->thick_mm;
    return (1.0 - u - v) * s->vthick[s->idx[3 * t]] + u * s->vthick[s->idx[3 * t + 1]] +
           v * s->vthick[s->idx[3 * t + 2]];
}

/* Texture coordinates of barycentric (u, v) on triangle t. */
static void tex_at(const orc_scene *s, int32_t t, double u, double v, double st[2])
{
    const double *q0 = s->uv + 2 * s->idx[3 * t], *q1 = s->uv + 2 * s->idx[3 * t + 1],
                 *q2 = s->uv + 2 * s->idx[3 * t + 2];
    for (int a = 0; a < 2; ++a) st[a] = (1.0 - u - v) * q0[a] + u * q1[a] + v * q2[a];
}

static int32_t clampi(double x, int32_t n)
{
    return x < 0.0 ? 0 : (x > (double)(n - 1) ? n - 1 : (int32_t)x);
}

/* Distribution maps (Sec. 6; texture coordinates of the hit, Sec. 3.1): the
 * texel under the hit gives the material; the thickness table, when there
 * is one, is interpolated bilinearly between texel centres. */
void orc_pane_at(const orc_scene *s, int32_t t, double u, double v, int32_t *material, double *thick_mm)
{
    int32_t m = s->mat[t];
    *material = m;
    int32_t mp = s->mats[m].map;
    if (mp < 0) {
        *thick_mm = thickness_at(s, t, u, v);
        return;
    }
    const omap *M = &s->maps[mp];
    double st[2];
    tex_at(s, t, u, v, st);
    *material = M->material[clampi(floor(st[1] * M->H), M->H) * M->W + clampi(floor(st[0] * M->W), M->W)];
    if (!M->thick) {
        *thick_mm = thickness_at(s, t, u, v);
        return;
    }
    double xs = st[0] * M->W - 0.5, ys = st[1] * M->H - 0.5;
    double x0 = floor(xs), y0 = floor(ys), fx = xs - x0, fy = ys - y0;
    int32_t xa = clampi(x0, M->W), xb = clampi(x0 + 1.0, M->W), ya = clampi(y0, M->H), yb = clampi(y0 + 1.0, M->H);
    const double *T = M->thick;
    *thick_mm = (1.0 - fy) * ((1.0 - fx) * T[ya * M->W + xa] + fx * T[ya * M->W + xb]) +
                fy * ((1.0 - fx) * T[yb * M->W + xa] + fx * T[yb * M->W + xb]);
}

/* Per-render material values at the render wavelengths. */
typedef struct {
    int32_t nl;
    double *lam, *rho, *n, *k, *tint, *E, *Lsky; /* rho/n/k/tint are [n_mat][nl] */
    double *nref, *sigma;                        /* [n_mat]: bubbly panes */
} spectra;

/* Sun transmittance along x + t * sun (t > teps, t unbounded): zero if any
 * opaque triangle is crossed, else the product of the slab transmittances of
 * every pane crossed (Sec. 3.1 shadow rays; eq. (3)). */
/* Event signatures (a debug aid, independent of the transport): the output
 * function of SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) applied to a packed event
 * word kind << 56 | vertex << 48 | x. */
static uint64_t event_hash(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Sun transmittance (below).  ev (may be NULL) receives, for the event
 * signature, -1 if the ray is occluded, else the number of panes crossed,
 * and ev_panes the sum of the hashes of 3 << 56 | triangle over them. */
static double shadow_T(const orc_scene *s, const spectra *sp, int use_bvh, const double *x,
                       int32_t skip, int li, double lambda_nm, int *ev, uint64_t *ev_panes,
                       const orc_render_params *pb_p, double pb_e, double *pb_s)
{
    double T = 1.0;
    int n_panes = 0;
    uint64_t pane_sum = 0;
    if (ev) *ev = 0;
    if (ev_panes) *ev_panes = 0;
    const double *d = s->sun;
    int32_t stack[256];
    int top = 0;
    if (s->nt == 0) return 1.0;
    if (use_bvh) stack[top++] = 0;
    int32_t brute = use_bvh ? -1 : 0;
    for (;;) {
        int32_t first, count;
        if (brute >= 0) {
            if (brute >= s->nt) break;
            first = brute; count = 1; brute++;
        } else {
            if (top == 0) break;
            const onode *n = &s->nodes[stack[--top]];
            if (!box_overlap(n, x, d, s->teps, INFINITY)) continue;
            if (n->left >= 0) { stack[top++] = n->left; stack[top++] = n->right; continue; }
            first = n->first; count = n->count;
        }
        for (int32_t i = first; i < first + count; ++i) {
            int32_t t = use_bvh ? s->order[i] : i;
            if (t == skip) continue;
            double tt, u, v;
            if (!tri_hit(s, t, x, d, &tt, &u, &v) || !(tt > s->teps)) continue;
            const omat *m = &s->mats[s->mat[t]];
            if (m->type == ORC_LAMBERT) {
                if (ev) *ev = -1;
                return 0.0;
            }
            ++n_panes;
            pane_sum += event_hash(3ULL << 56 | (uint32_t)t);
            double R, Tr;
            double c = fabs(dot3(d, s->ng + 3 * t));
            int32_t mi;
            double thick;
            orc_pane_at(s, t, u, v, &mi, &thick);
            if (pb_s) {
                double xh[3];
                for (int a = 0; a < 3; ++a) xh[a] = x[a] + tt * d[a];
                double alpha = 4.0 * PI * sp->k[mi * sp->nl + li] / (lambda_nm * 1e-6) + sp->tint[mi * sp->nl + li] +
                               sp->sigma[mi];
                *pb_s += pb_p->prec_rel + pane_sensitivity(pb_p, s, t, u, v, hit_error(pb_p, pb_e, tt, c, xh), c,
                                                           sp->n[mi * sp->nl + li], alpha);
            }
            /* Reading: toward the delta sun only the unscattered (ballistic)
             * light of a bubbly pane counts, so the bubbles' extinction adds
             * to the absorption of the slab. */
            orc_slab(c, lambda_nm, thick, sp->n[mi * sp->nl + li], sp->k[mi * sp->nl + li],
                     sp->tint[mi * sp->nl + li] + sp->sigma[mi], &R, &Tr);
            T *= Tr;
        }
    }
    if (ev) *ev = n_panes;
    if (ev_panes) *ev_panes = pane_sum;
    return T;
}

void orc_intersect(const orc_scene *s, int32_t use_bvh, int64_t m, const double *o, const double *dir,
                   const int32_t *skip, double *t, int32_t *tri, double *u, double *v)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        ohit h = closest(s, use_bvh, o + 3 * i, dir + 3 * i, skip ? skip[i] : -1);
        t[i] = h.t; tri[i] = h.tri; u[i] = h.u; v[i] = h.v;
    }
}

/* ------------------------------------------------------------------------- */
/* Tables                                                                     */
/* ------------------------------------------------------------------------- */
/* Reading: tables are linearly interpolated to the render wavelengths and
 * held constant beyond their ends. */
static double interp_tab(const orc_scene *s, const double *ys, double x)
{
    const double *xs = s->tab_lambda;
    int n = s->n_tab;
    if (n == 1 || x <= xs[0]) return ys[0];
    if (x >= xs[n - 1]) return ys[n - 1];
    int i = 0;
    while (xs[i + 1] < x) ++i;
    double w = (x - xs[i]) / (xs[i + 1] - xs[i]);
    return (1.0 - w) * ys[i] + w * ys[i + 1];
}

static void spectra_make(const orc_scene *s, const orc_render_params *p, spectra *sp)
{
    int nl = p->n_lambda, nm = s->n_mat;
    sp->nl = nl;
    sp->lam = (double *)malloc(sizeof(double) * (size_t)nl);
    sp->rho = (double *)calloc((size_t)(nm * nl + 1), sizeof(double));
    sp->n = (double *)calloc((size_t)(nm * nl + 1), sizeof(double));
    sp->k = (double *)calloc((size_t)(nm * nl + 1), sizeof(double));
    sp->tint = (double *)calloc((size_t)(nm * nl + 1), sizeof(double));
    sp->E = (double *)malloc(sizeof(double) * (size_t)nl);
    sp->Lsky = (double *)malloc(sizeof(double) * (size_t)nl);
    sp->nref = (double *)calloc((size_t)(nm + 1), sizeof(double));
    sp->sigma = (double *)calloc((size_t)(nm + 1), sizeof(double));
    for (int m = 0; m < nm; ++m) {
        const omat *mm = &s->mats[m];
        /* Reading: inside a bubbly pane the walk uses the pane's index at
         * 560 nm (R1 interpolation of its table). */
        sp->nref[m] = mm->n ? interp_tab(s, mm->n, 560.0) : 1.0;
        if (mm->type == ORC_GLASS_BUBBLY) sp->sigma[m] = orc_bubble_sigma(mm->density, mm->rmin_um, mm->rmax_um);
    }
    for (int i = 0; i < nl; ++i) {
        double x = p->lambda_nm[i];
        sp->lam[i] = x;
        sp->E[i] = interp_tab(s, s->sun_E, x);
        sp->Lsky[i] = interp_tab(s, s->sky_L, x);
        for (int m = 0; m < nm; ++m) {
            const omat *mm = &s->mats[m];
            if (mm->albedo) sp->rho[m * nl + i] = interp_tab(s, mm->albedo, x);
            if (mm->n) sp->n[m * nl + i] = interp_tab(s, mm->n, x);
            if (mm->k) sp->k[m * nl + i] = interp_tab(s, mm->k, x);
            if (mm->tint) sp->tint[m * nl + i] = interp_tab(s, mm->tint, x);
        }
    }
}

static void spectra_free(spectra *sp)
{
    free(sp->lam); free(sp->rho); free(sp->n); free(sp->k); free(sp->tint); free(sp->E); free(sp->Lsky);
    free(sp->nref); free(sp->sigma);
}

/* ------------------------------------------------------------------------- */
/* Path tracing                                                               */
/* ------------------------------------------------------------------------- */
typedef struct {
    double eye[3], f[3], r[3], u[3];
    double th, aspect, oh;
} camera;

static void camera_make(const orc_render_params *p, camera *c)
{
    for (int a = 0; a < 3; ++a) c->eye[a] = p->eye[a];
    sub3(p->target, p->eye, c->f);
    normalize3(c->f);
    cross3(c->f, p->up, c->r);
    normalize3(c->r);
    cross3(c->r, c->f, c->u);
    c->th = tan(0.5 * p->vfov_deg * PI / 180.0);
    c->aspect = (double)p->W / (double)p->H;
    c->oh = 0.5 * p->ortho_height;
}

/* Reading: image point (x, y) = ((i + u0) / W, (j + u1) / H), row j counted
 * from the top.  Pinhole: from the eye through the image plane at unit
 * distance; orthographic: rays orthogonal to the image plane (Sec. 3.1). */
static void camera_ray(const orc_render_params *p, const camera *c, int i, int j, const double *u,
                       double *o, double *d)
{
    double x = (i + u[0]) / p->W, y = (j + u[1]) / p->H;
    double a = 2.0 * x - 1.0, b = 1.0 - 2.0 * y;
    if (p->projection == 1) {
        for (int k = 0; k < 3; ++k) {
            o[k] = c->eye[k] + a * c->oh * c->aspect * c->r[k] + b * c->oh * c->u[k];
            d[k] = c->f[k];
        }
        return;
    }
    for (int k = 0; k < 3; ++k) {
        o[k] = c->eye[k];
        d[k] = c->f[k] + a * c->th * c->aspect * c->r[k] + b * c->th * c->u[k];
    }
    normalize3(d);
}

/* Reading: tangent basis about unit n from a fixed generic axis h = (1, 2,
 * 3) / sqrt(14): t1 = normalize(h x n), t2 = n x t1.  It is continuous for
 * every normal except +-h, so axis-aligned and vertical faces (the common
 * case in architecture) never sit on the switch of a branch-based basis,
 * where the choice would hang on the sign of a rounding residue. */
static void onb(const double *n, double *t1, double *t2)
{
    const double h[3] = {0.2672612419124244, 0.5345224838248488, 0.8017837257372732};
    cross3(h, n, t1);
    normalize3(t1);
    cross3(n, t1, t2);
}

/* A stored photon of the caustic map, and the map hashed by cells of side r. */
typedef struct {
    double x[3], n[3], phi;
    int32_t j;
} ophot;

typedef struct {
    int64_t n;
    ophot *ph;
    uint32_t mask;
    int64_t *start;   /* [buckets + 1] */
    int64_t *idx;     /* photon indices by bucket */
    double r, lo[3];
} ophmap;

typedef struct {
    const orc_scene *s;
    const orc_render_params *p;
    const spectra *sp;
    camera cam;
    const ophmap *ph;
} rctx;

void orc_camera_ray(const orc_render_params *p, int32_t i, int32_t j, double u0, double u1,
                    double o[3], double d[3])
{
    camera c;
    camera_make(p, &c);
    double u[2] = {u0, u1};
    camera_ray(p, &c, i, j, u, o, d);
}

/* Reading: cosine-weighted bounce (Malley's method: uniform disk point
 * lifted to the hemisphere) in the basis of onb(). */
static void cosine_dir(const double *ns, double u1, double u2, double *d)
{
    double t1[3], t2[3];
    onb(ns, t1, t2);
    double rr = sqrt(u1), phi = 2.0 * PI * u2, lz = sqrt(1.0 - u1);
    double lx = rr * cos(phi), ly = rr * sin(phi);
    for (int a = 0; a < 3; ++a) d[a] = lx * t1[a] + ly * t2[a] + lz * ns[a];
}

void orc_cosine_dir(const double n[3], double u1, double u2, double d[3]) { cosine_dir(n, u1, u2, d); }

/* Reading: the surrogate's transmitted direction is d plus a 2-D Gaussian
 * offset of standard deviation w per tangent axis (Box-Muller on u1, u2) in
 * the basis of onb(d), normalised. */
void orc_lobe_dir(const double d[3], double w, double u1, double u2, double out[3])
{
    double t1[3], t2[3];
    onb(d, t1, t2);
    double g = sqrt(-2.0 * log1p(-u1)), phi = 2.0 * PI * u2;
    double g1 = g * cos(phi), g2 = g * sin(phi);
    for (int a = 0; a < 3; ++a) out[a] = d[a] + w * (g1 * t1[a] + g2 * t2[a]);
    normalize3(out);
}

/* Reading: a lobe sample that would leave through the entry side of the
 * pane (the sign of its component along the face normal ng differs from the
 * incoming ray's) is mirrored across the pane's plane, so that transmitted
 * light always continues on the far side, as every transmitted exit of the
 * photon walk does. */
void orc_lobe_transmit(const double d[3], const double ng[3], double w, double u1, double u2, double out[3])
{
    orc_lobe_dir(d, w, u1, u2, out);
    double dn = dot3(out, ng);
    if (dn * dot3(d, ng) < 0.0)
        for (int a = 0; a < 3; ++a) out[a] -= 2.0 * dn * ng[a];
}

/* Slab frame of a hit: z along the face normal on the far side of the
 * incoming ray, x along the ray's component in the face (the onb() axis
 * when the ray meets the face head-on), y = z x x. */
void orc_slab_to_world(const double d[3], const double ng[3], const double a[3], double out[3])
{
    double nz[3], ex[3], ey[3], t2[3];
    double dn = dot3(d, ng);
    for (int i = 0; i < 3; ++i) nz[i] = dn > 0.0 ? ng[i] : -ng[i];
    double c = fabs(dn);
    for (int i = 0; i < 3; ++i) ex[i] = d[i] - c * nz[i];
    double len = sqrt(dot3(ex, ex));
    if (len > 1e-7) {
        for (int i = 0; i < 3; ++i) ex[i] /= len;
    } else {
        onb(nz, ex, t2);
    }
    cross3(nz, ex, ey);
    for (int i = 0; i < 3; ++i) out[i] = a[0] * ex[i] + a[1] * ey[i] + a[2] * nz[i];
    normalize3(out);
}

/* Evaluation of a bubbly-pane vertex: the mode, after the error-table check
 * of the fallback mode (cell value above the bound -> exact walk). */
static int bubbly_mode(const orc_render_params *p, const omat *mm, double cos_i, double d)
{
    if (p->btdf_mode != ORC_BTDF_FALLBACK) return p->btdf_mode;
    const int nc = p->err_dims[0], nd = p->err_dims[1], nr = p->err_dims[2];
    int ic = (int)(cos_i * nc);
    int id = (int)((d - ORC_ERR_D_LO) / (ORC_ERR_D_HI - ORC_ERR_D_LO) * nd);
    int ir = (int)(mm->density / ORC_ERR_RHO_HI * nr);
    ic = ic < 0 ? 0 : (ic >= nc ? nc - 1 : ic);
    id = id < 0 ? 0 : (id >= nd ? nd - 1 : id);
    ir = ir < 0 ? 0 : (ir >= nr ? nr - 1 : ir);
    double e = p->err_table[(((int64_t)mm->pane_id * nc + ic) * nd + id) * nr + ir];
    return e > p->err_bound ? ORC_BTDF_EXACT : ORC_BTDF_SURROGATE;
}

/* The network at one vertex; with bnd (BF16 mode only), also the bound of
 * orc_mlp_bf16_bound for cos and thickness inputs off by e_cos and e_d. */
static void surrogate_eval(const orc_render_params *p, const omat *mm, double cos_i, double lambda, double d,
                           double out[3], double e_cos, double e_d, double *bnd)
{
    double tup[4] = {cos_i, lambda, d, mm->density};
    int32_t pane = mm->pane_id;
    if (p->mlp_bf16 && bnd) orc_mlp_bf16_bound(p->mlp_params, tup, pane, e_cos, e_d, out, bnd);
    else if (p->mlp_bf16) orc_mlp_forward_bf16(p->mlp_params, p->mlp_n_panes, 1, tup, &pane, out);
    else orc_mlp_forward(p->mlp_params, p->mlp_n_panes, 1, tup, &pane, out);
}

/* ------------------------------------------------------------------------- */
/* Caustic photon map (photon mapping, Sec. 3.2)                              */
/* ------------------------------------------------------------------------- */
#define PHOTON_TAG 0xFFFFFFF0u   /* sample word of the photons' draws */

static uint32_t ph_hash(int64_t ix, int64_t iy, int64_t iz, uint32_t mask)
{
    return (((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u)) & mask;
}

static void ph_cell(const ophmap *m, const double *x, int64_t c[3])
{
    for (int a = 0; a < 3; ++a) c[a] = (int64_t)floor((x[a] - m->lo[a]) / m->r);
}

/* One photon: the sun's photon pid leaves the emission square (centre c,
 * half sides e1 and e2) toward -sun with one render wavelength, follows the
 * panes for up to max_depth vertices, and is stored (returns 1) where it
 * first meets a Lambert surface if a pane has turned it: a reflection at
 * clear glass (probability R / (R + T), weight R + T), or at a bubbly pane an
 * entry reflection, an exit back through the entry face or a bubble met on
 * the walk (weight exp(-alpha L)).  Light that goes straight through (clear
 * transmission, unscattered bubbly transmission) is the shadow rays'. */
static int trace_photon(const rctx *c, uint32_t pid, const double cen[3], const double e1[3], const double e2[3],
                        double power, ophot *out)
{
    const orc_scene *s = c->s;
    const orc_render_params *p = c->p;
    const spectra *sp = c->sp;
    double u[4], o[3], d[3];
    draw4(p->seed, p->job_id, pid, PHOTON_TAG, -1, 0, u);
    double a = 2.0 * u[0] - 1.0, b = 2.0 * u[1] - 1.0;
    int j = (int)(u[2] * sp->nl);
    if (j > sp->nl - 1) j = sp->nl - 1;
    for (int q = 0; q < 3; ++q) {
        o[q] = cen[q] + a * e1[q] + b * e2[q];
        d[q] = -s->sun[q];
    }
    double lambda = sp->lam[j];
    double phi = sp->E[j] * power;
    int turned = 0;
    int32_t skip = -1;
    for (int vtx = 0; vtx < p->max_depth; ++vtx) {
        ohit h = closest(s, p->use_bvh, o, d, skip);
        if (h.tri < 0 || !(phi > 0.0)) return 0;
        double x[3];
        for (int q = 0; q < 3; ++q) x[q] = o[q] + h.t * d[q];
        const double *ng = s->ng + 3 * h.tri;
        double cos_i = fabs(dot3(d, ng));
        int32_t mi = s->mat[h.tri];
        const omat *mm = &s->mats[mi];
        if (mm->type == ORC_LAMBERT) {
            if (!turned) return 0;
            double sg = dot3(ng, d) > 0.0 ? -1.0 : 1.0;
            for (int q = 0; q < 3; ++q) {
                out->x[q] = x[q];
                out->n[q] = sg * ng[q];
            }
            out->phi = phi;
            out->j = j;
            return 1;
        }
        if (mm->type == ORC_GLASS) {
            int32_t me;
            double thick, R, T;
            orc_pane_at(s, h.tri, h.u, h.v, &me, &thick);
            orc_slab(cos_i, lambda, thick, sp->n[me * sp->nl + j], sp->k[me * sp->nl + j], sp->tint[me * sp->nl + j],
                     &R, &T);
            draw4(p->seed, p->job_id, pid, PHOTON_TAG, vtx, 0, u);
            if (R + T > 0.0 && u[0] < R / (R + T)) {
                double dn = dot3(d, ng);
                for (int q = 0; q < 3; ++q) d[q] -= 2.0 * dn * ng[q];
                turned = 1;
            }
            phi *= R + T;
        } else {
            double thick = thickness_at(s, h.tri, h.u, h.v);
            orc_walk_stream st = {p->seed, pid, PHOTON_TAG, p->job_id, (uint32_t)vtx, 1};
            double ue[4], Rs, Rp;
            orc_walk_draw(&st, 0, 0, ue);
            int pol = ue[1] < 0.5 ? 0 : 1;
            orc_fresnel(cos_i, sp->n[mi * sp->nl + j], sp->k[mi * sp->nl + j], &Rs, &Rp);
            if (ue[0] < (pol == 0 ? Rs : Rp)) {
                double dn = dot3(d, ng);
                for (int q = 0; q < 3; ++q) d[q] -= 2.0 * dn * ng[q];
                turned = 1;
            } else {
                orc_walk_out wo;
                orc_bubbly_walk(&st, cos_i, thick, sp->sigma[mi], sp->nref[mi], pol, &wo);
                if (wo.kind == 0) return 0;
                double nd[3];
                orc_slab_to_world(d, ng, wo.dir, nd);
                for (int q = 0; q < 3; ++q) d[q] = nd[q];
                if (wo.kind == 1 || wo.bubbles > 0) turned = 1;
                double alpha = 4.0 * PI * sp->k[mi * sp->nl + j] / (lambda * 1e-6) + sp->tint[mi * sp->nl + j];
                phi *= exp(-alpha * wo.L);
            }
        }
        for (int q = 0; q < 3; ++q) o[q] = x[q];
        skip = h.tri;
    }
    return 0;
}

/* The first pass: every photon traced, the stored ones kept in photon order
 * and hashed by the cells of side r. */
static void photon_map_build(const rctx *c, ophmap *m)
{
    const orc_scene *s = c->s;
    const orc_render_params *p = c->p;
    memset(m, 0, sizeof(*m));
    if (p->photons <= 0) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < 3 * (int64_t)s->nt; ++i)
        for (int a = 0; a < 3; ++a) {
            double x = s->pos[3 * s->idx[i] + a];
            lo[a] = fmin(lo[a], x);
            hi[a] = fmax(hi[a], x);
        }
    double cen[3], rad = 0.0, e1[3], e2[3], h[3] = {0.2672612419124244, 0.5345224838248488, 0.8017837257372732};
    for (int a = 0; a < 3; ++a) {
        cen[a] = 0.5 * (lo[a] + hi[a]);
        rad += 0.25 * (hi[a] - lo[a]) * (hi[a] - lo[a]);
    }
    rad = sqrt(rad) + 1e-6;
    cross3(h, s->sun, e1);
    normalize3(e1);
    cross3(s->sun, e1, e2);
    double c0[3], a1[3], a2[3];
    for (int a = 0; a < 3; ++a) {
        c0[a] = cen[a] + 2.0 * rad * s->sun[a];
        a1[a] = rad * e1[a];
        a2[a] = rad * e2[a];
    }
    double power = 4.0 * rad * rad * (double)c->sp->nl / (double)p->photons;
    int64_t N = p->photons;
    ophot *all = (ophot *)malloc(sizeof(ophot) * (size_t)N);
    char *kept = (char *)calloc((size_t)N, 1);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < N; ++q) kept[q] = (char)trace_photon(c, (uint32_t)q, c0, a1, a2, power, &all[q]);
    int64_t n = 0;
    for (int64_t q = 0; q < N; ++q)
        if (kept[q]) all[n++] = all[q];
    free(kept);
    m->n = n;
    m->ph = all;
    m->r = p->photon_radius;
    for (int a = 0; a < 3; ++a) m->lo[a] = lo[a];
    uint32_t buckets = 1024;
    while (buckets < 2 * (uint64_t)n && buckets < (1u << 24)) buckets <<= 1;
    m->mask = buckets - 1;
    m->start = (int64_t *)calloc((size_t)buckets + 1, sizeof(int64_t));
    m->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t cc[3];
    for (int64_t q = 0; q < n; ++q) {
        ph_cell(m, m->ph[q].x, cc);
        m->start[ph_hash(cc[0], cc[1], cc[2], m->mask) + 1]++;
    }
    for (uint32_t b = 0; b < buckets; ++b) m->start[b + 1] += m->start[b];
    int64_t *fill = (int64_t *)calloc((size_t)buckets, sizeof(int64_t));
    for (int64_t q = 0; q < n; ++q) {
        ph_cell(m, m->ph[q].x, cc);
        uint32_t b = ph_hash(cc[0], cc[1], cc[2], m->mask);
        m->idx[m->start[b] + fill[b]++] = q;
    }
    free(fill);
}

static void photon_map_free(ophmap *m)
{
    free(m->ph);
    free(m->start);
    free(m->idx);
}

/* Density estimate of the caustic light at x (surface side normal ns) for
 * wavelength j: the stored power of the photons of that wavelength within r
 * whose arrival side's normal is within 0.9 (cosine) of ns, over pi r^2.
 * Each cell of the 27 around x is read once (cells may share a bucket). */
static double photon_gather(const ophmap *m, const double *x, const double *ns, int j)
{
    int64_t cc[3];
    ph_cell(m, x, cc);
    uint32_t seen[27];
    int n_seen = 0;
    double sum = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                uint32_t b = ph_hash(cc[0] + dx, cc[1] + dy, cc[2] + dz, m->mask);
                int dup = 0;
                for (int q = 0; q < n_seen; ++q) dup |= seen[q] == b;
                if (dup) continue;
                seen[n_seen++] = b;
                for (int64_t k = m->start[b]; k < m->start[b + 1]; ++k) {
                    const ophot *ph = &m->ph[m->idx[k]];
                    if (ph->j != j) continue;
                    double e[3];
                    sub3(ph->x, x, e);
                    if (!(dot3(e, e) < m->r * m->r)) continue;
                    if (!(dot3(ph->n, ns) > 0.9)) continue;
                    sum += ph->phi;
                }
            }
    return sum / (PI * m->r * m->r);
}

static int params_ok(const orc_scene *s, const orc_render_params *p);

int64_t orc_photon_map(const orc_scene *s, const orc_render_params *p, double *out)
{
    if (!params_ok(s, p)) return -1;
    spectra sp;
    spectra_make(s, p, &sp);
    rctx c = {s, p, &sp, {{0}}, NULL};
    ophmap m;
    photon_map_build(&c, &m);
    if (out)
        for (int64_t q = 0; q < m.n; ++q) {
            for (int a = 0; a < 3; ++a) {
                out[8 * q + a] = m.ph[q].x[a];
                out[8 * q + 3 + a] = m.ph[q].n[a];
            }
            out[8 * q + 6] = m.ph[q].phi;
            out[8 * q + 7] = m.ph[q].j;
        }
    int64_t n = m.n;
    photon_map_free(&m);
    spectra_free(&sp);
    return n;
}

/* One (pixel, sample, wavelength) path estimate.  ev (may be NULL): the
 * path's events are added to *ev (event signature); pb (may be NULL): the
 * single-precision error bound of its contributions is added to *pb (see
 * orc_render_params). */
static double path_radiance(const rctx *c, int i, int j, int smp, int li, uint64_t *ev, double *pb)
{
    const orc_scene *s = c->s;
    const orc_render_params *p = c->p;
    const spectra *sp = c->sp;
    uint32_t pixel = (uint32_t)(j * p->W + i);
    double u[4], o[3], d[3];
    draw4(p->seed, p->job_id, pixel, (uint32_t)smp, -1, 0, u);
    camera_ray(p, &c->cam, i, j, u, o, d);
    double lambda = sp->lam[li];
    double beta = 1.0, L = 0.0;
    int32_t skip = -1;
    /* single-precision bound: error of the current ray origin (a camera
     * origin is rounded once) and relative error of the path weight */
    double epos = p->prec_eps * fmax(fmax(fabs(o[0]), fabs(o[1])), fabs(o[2]));
    double sbeta = 0.0;
    /* extra error of the current direction (radians) beyond its rounding, set
     * where a bubbly vertex chose it: moves the next hit by edir * t */
    double edir = 0.0;
    /* Reading: vertices 0 .. max_depth-1 are shaded; the last one does its
     * light sum but traces no continuation; no Russian roulette. */
    for (int vtx = 0; vtx < p->max_depth; ++vtx) {
        ohit h = closest(s, p->use_bvh, o, d, skip);
        if (ev && beta != 0.0)
            *ev += event_hash(1ULL << 56 | (uint64_t)vtx << 48 | (uint64_t)(uint32_t)smp << 32 |
                              (uint32_t)(h.tri + 1));
        if (h.tri < 0) {
            /* Reading: every escaping ray sees the uniform sky; the sun is a
             * delta light reached only through the shadow rays. */
            L += beta * sp->Lsky[li];
            if (pb) *pb += fabs(beta * sp->Lsky[li]) * (sbeta + p->prec_rel);
            break;
        }
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = o[a] + h.t * d[a];
        draw4(p->seed, p->job_id, pixel, (uint32_t)smp, vtx, 0, u);
        int32_t mi = s->mat[h.tri];
        const double *ng = s->ng + 3 * h.tri;
        if (pb) {
            epos = hit_error(p, epos + edir * h.t, h.t, fabs(dot3(d, ng)), x);
            edir = 0.0;
        }
        if (s->mats[mi].type == ORC_LAMBERT) {
            double ns[3] = {ng[0], ng[1], ng[2]};
            if (dot3(ns, d) > 0.0) { ns[0] = -ns[0]; ns[1] = -ns[1]; ns[2] = -ns[2]; }
            double rho = sp->rho[mi * sp->nl + li];
            double cs = dot3(ns, s->sun);
            if (cs > 0.0) {
                int sev;
                double s_sh = 0.0;
                uint64_t spanes;
                double T = shadow_T(s, sp, p->use_bvh, x, h.tri, li, lambda, &sev, &spanes, p, epos,
                                    pb ? &s_sh : NULL);
                if (ev && beta * rho != 0.0)
                    *ev += event_hash(2ULL << 56 | (uint64_t)vtx << 48 | (sev < 0 ? 0xFFFFULL : (uint64_t)sev)) +
                           (sev > 0 ? spanes : 0);
                /* eq. (3): Lambert BRDF rho / pi times E_sun cos(theta). */
                L += beta * rho / PI * sp->E[li] * cs * T;
                if (pb)
                    *pb += fabs(beta * rho / PI * sp->E[li] * cs * T) *
                           (sbeta + 3.0 * p->prec_rel + p->prec_ceps / cs + s_sh);
            }
            if (c->ph) {
                /* caustic photon map: rho / pi times the density estimate of
                 * the turned sunlight arriving on this side */
                double Lc = beta * rho / PI * photon_gather(c->ph, x, ns, li);
                L += Lc;
                if (pb) *pb += fabs(Lc) * (sbeta + 3.0 * p->prec_rel);
            }
            if (vtx == p->max_depth - 1) break;
            /* The cosine/pdf ratio of the bounce cancels pi, so the path
             * weight is multiplied by the albedo. */
            cosine_dir(ns, u[1], u[2], d);
            beta *= rho;
            sbeta += p->prec_rel;
        } else if (s->mats[mi].type == ORC_GLASS_BUBBLY) {
            /* Bubbly pane (air micro-particles, Sec. 1; scattering, Sec. 6). */
            if (vtx == p->max_depth - 1) break;
            const omat *mm = &s->mats[mi];
            double cos_i = fabs(dot3(d, ng));
            if (pb) {
                double alpha = 4.0 * PI * sp->k[mi * sp->nl + li] / (lambda * 1e-6) + sp->tint[mi * sp->nl + li];
                sbeta += p->prec_rel + glass_sensitivity(p, s, h.tri, epos, cos_i, sp->n[mi * sp->nl + li], alpha);
            }
            double thick = thickness_at(s, h.tri, h.u, h.v);
            if (bubbly_mode(p, mm, cos_i, thick) == ORC_BTDF_EXACT) {
                /* Exact walk: entry interface at this wavelength (eq. (1)),
                 * then the wavelength-independent walk inside; the weight is
                 * the absorption along the walk's length in glass. */
                orc_walk_stream st = {p->seed, pixel, (uint32_t)smp, p->job_id, (uint32_t)vtx, 1};
                double ue[4], Rs, Rp;
                orc_walk_draw(&st, 0, 0, ue);
                int pol = ue[1] < 0.5 ? 0 : 1;
                orc_fresnel(cos_i, sp->n[mi * sp->nl + li], sp->k[mi * sp->nl + li], &Rs, &Rp);
                if (ue[0] < (pol == 0 ? Rs : Rp)) {
                    double dn = dot3(d, ng);
                    for (int a = 0; a < 3; ++a) d[a] -= 2.0 * dn * ng[a];
                } else {
                    orc_walk_out wo;
                    orc_bubbly_walk(&st, cos_i, thick, sp->sigma[mi], sp->nref[mi], pol, &wo);
                    if (wo.kind == 0) break;
                    double alpha = 4.0 * PI * sp->k[mi * sp->nl + li] / (lambda * 1e-6) + sp->tint[mi * sp->nl + li];
                    double nd[3];
                    orc_slab_to_world(d, ng, wo.dir, nd);
                    for (int a = 0; a < 3; ++a) d[a] = nd[a];
                    beta *= exp(-alpha * wo.L);
                    if (pb) {
                        /* FP32 walk: each free flight's length and the running
                         * sums carry a few roundings (2 prec_rel per flight);
                         * every length scales with the thickness, which is
                         * off by |grad d| epos; the exit direction carries the
                         * flights' rounding, magnified near grazing exit */
                        double nf = (double)(wo.n_events + 1);
                        sbeta += alpha * wo.L * (2.0 * nf * p->prec_rel + thickness_grad(s, h.tri) * epos / thick);
                        edir += 4.0 * nf * p->prec_rel / fmax(fabs(wo.dir[2]), 1e-3);
                    }
                }
            } else {
                /* Surrogate: (R, T) at this wavelength; reflect with
                 * probability R / (R + T), else leave through the
                 * transmitted lobe, whose width is taken at 560 nm so that
                 * every wavelength of the path keeps one direction. */
                double y[3], yr[3], by[3], byr[3];
                const double e_d = pb ? thickness_grad(s, h.tri) * epos : 0.0;
                surrogate_eval(p, mm, cos_i, lambda, thick, y, p->prec_ceps, e_d, pb ? by : NULL);
                surrogate_eval(p, mm, cos_i, 560.0, thick, yr, p->prec_ceps, e_d, pb ? byr : NULL);
                if (u[0] < y[0] / (y[0] + y[1])) {
                    double dn = dot3(d, ng);
                    for (int a = 0; a < 3; ++a) d[a] -= 2.0 * dn * ng[a];
                } else {
                    double nd[3];
                    orc_lobe_transmit(d, ng, yr[2], u[1], u[2], nd);
                    for (int a = 0; a < 3; ++a) d[a] = nd[a];
                    /* the lobe offset is w g with g = sqrt(-2 ln(1 - u1)) */
                    if (pb && p->mlp_bf16) edir += byr[2] * sqrt(-2.0 * log1p(-u[1]));
                }
                beta *= y[0] + y[1];
                if (pb && p->mlp_bf16) sbeta += (by[0] + by[1]) / (y[0] + y[1]) + p->prec_rel;
            }
        } else {
            /* Glass pane as a thin slab (Sec. 6 thickness map): the path
             * reflects with probability R/(R+T), else passes straight
             * through; the weight is R + T. */
            double cos_i = fabs(dot3(d, ng));
            int32_t me;
            double thick;
            orc_pane_at(s, h.tri, h.u, h.v, &me, &thick);
            if (pb && vtx < p->max_depth - 1) {
                double alpha = 4.0 * PI * sp->k[me * sp->nl + li] / (lambda * 1e-6) + sp->tint[me * sp->nl + li];
                sbeta += p->prec_rel + pane_sensitivity(p, s, h.tri, h.u, h.v, epos, cos_i, sp->n[me * sp->nl + li],
                                                        alpha);
            }
            double R, T;
            orc_slab(cos_i, lambda, thick, sp->n[me * sp->nl + li], sp->k[me * sp->nl + li],
                     sp->tint[me * sp->nl + li], &R, &T);
            if (vtx == p->max_depth - 1) break;
            if (R + T > 0.0 && u[0] < R / (R + T)) {
                double dn = dot3(d, ng);
                for (int a = 0; a < 3; ++a) d[a] -= 2.0 * dn * ng[a];
            }
            beta *= R + T;
        }
        /* Energy threshold of Sec. 3.1 (off when 0). */
        if (beta < p->beta_threshold) break;
        for (int a = 0; a < 3; ++a) o[a] = x[a];
        skip = h.tri;
    }
    return L;
}

static int params_ok(const orc_scene *s, const orc_render_params *p)
{
    if (!s || !p || p->W < 1 || p->H < 1 || p->spp < 1 || p->max_depth < 1 || p->n_lambda < 1 ||
        !p->lambda_nm)
        return 0;
    if (p->btdf_mode < ORC_BTDF_EXACT || p->btdf_mode > ORC_BTDF_FALLBACK) return 0;
    if (p->photons < 0 || (p->photons > 0 && !(p->photon_radius > 0.0))) return 0;
    for (int m = 0; m < s->n_mat; ++m) {
        const omat *mm = &s->mats[m];
        if (mm->type != ORC_GLASS_BUBBLY || p->btdf_mode == ORC_BTDF_EXACT) continue;
        if (!p->mlp_params || mm->pane_id < 0 || mm->pane_id >= p->mlp_n_panes) return 0;
        if (p->btdf_mode == ORC_BTDF_FALLBACK &&
            (!p->err_table || p->err_dims[0] < 1 || p->err_dims[1] < 1 || p->err_dims[2] < 1))
            return 0;
    }
    return 1;
}

/* Reading: trapezoid weights in nm over the render grid (1 for a single
 * wavelength), no normalising constant. */
static void trapezoid(int nl, const double *lam, double *w)
{
    if (nl == 1) { w[0] = 1.0; return; }
    for (int i = 0; i < nl; ++i) {
        double a = lam[i > 0 ? i - 1 : 0], b = lam[i < nl - 1 ? i + 1 : nl - 1];
        w[i] = 0.5 * (b - a);
    }
}

void orc_spec_to_xyz(int64_t npix, int32_t nl, const double *lam, const double *cmf,
                     const double *spec, double *xyz)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)nl);
    trapezoid(nl, lam, w);
    for (int64_t q = 0; q < npix; ++q)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int i = 0; i < nl; ++i) acc += w[i] * spec[q * nl + i] * cmf[3 * i + c];
            xyz[3 * q + c] = acc;
        }
    free(w);
}

static void pixel_spectrum(const rctx *c, int i, int j, int l0, int l1, double *out, uint64_t *ev, double *pb)
{
    for (int li = l0; li < l1; ++li) {
        double sum = 0.0, bound = 0.0;
        uint64_t e = 0;
        for (int smp = 0; smp < c->p->spp; ++smp)
            sum += path_radiance(c, i, j, smp, li, ev ? &e : NULL, pb ? &bound : NULL);
        out[li] = sum / c->p->spp;
        if (ev) ev[li] = e;
        if (pb) pb[li] = bound / c->p->spp;
    }
}

int orc_render(const orc_scene *s, const orc_render_params *p, double *spec, double *xyz)
{
    if (!params_ok(s, p) || !spec) return -1;
    spectra sp;
    spectra_make(s, p, &sp);
    rctx c = {s, p, &sp, {{0}}, NULL};
    camera_make(p, &c.cam);
    ophmap phm;
    photon_map_build(&c, &phm);
    if (p->photons > 0) c.ph = &phm;
    int nl = p->n_lambda;
    int B = p->n_bands < 1 ? 1 : (p->n_bands > nl ? nl : p->n_bands);
    int tile = p->tile > 0 ? p->tile : 16;
    int tx = (p->W + tile - 1) / tile, ty = (p->H + tile - 1) / tile;
    int64_t items = (int64_t)tx * ty * B;
    int64_t it0 = p->item_begin < 0 ? 0 : (p->item_begin > items ? items : p->item_begin);
    int64_t it1 = p->max_items > 0 && p->max_items < items - it0 ? it0 + p->max_items : items;
#ifdef _OPENMP
    if (p->n_threads > 0) omp_set_num_threads(p->n_threads);
#endif
    /* Work items = pixel tile x spectral band (Sec. 4, Sec. 5), pulled
     * dynamically by the threads (dynamic job balancing, Sec. 4).  Bands are
     * contiguous, the first nl mod B one wavelength larger. */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t it = it0; it < it1; ++it) {
        int band = (int)(it % B);
        int64_t tile_id = it / B;
        int bx = (int)(tile_id % tx), by = (int)(tile_id / tx);
        int base = nl / B, extra = nl % B;
        int l0 = band * base + (band < extra ? band : extra);
        int l1 = l0 + base + (band < extra ? 1 : 0);
        for (int j = by * tile; j < (by + 1) * tile && j < p->H; ++j)
            for (int i = bx * tile; i < (bx + 1) * tile && i < p->W; ++i)
                pixel_spectrum(&c, i, j, l0, l1, spec + ((int64_t)j * p->W + i) * nl,
                               p->events ? p->events + ((int64_t)j * p->W + i) * nl : NULL,
                               p->prec_bound ? p->prec_bound + ((int64_t)j * p->W + i) * nl : NULL);
    }
    if (xyz && p->cmf_xyz) orc_spec_to_xyz((int64_t)p->W * p->H, nl, p->lambda_nm, p->cmf_xyz, spec, xyz);
    photon_map_free(&phm);
    spectra_free(&sp);
    return 0;
}

int orc_render_pixels(const orc_scene *s, const orc_render_params *p, int64_t m, const int32_t *pixels,
                      double *spec)
{
    if (!params_ok(s, p) || !spec || !pixels) return -1;
    spectra sp;
    spectra_make(s, p, &sp);
    rctx c = {s, p, &sp, {{0}}, NULL};
    camera_make(p, &c.cam);
    ophmap phm;
    photon_map_build(&c, &phm);
    if (p->photons > 0) c.ph = &phm;
#ifdef _OPENMP
    if (p->n_threads > 0) omp_set_num_threads(p->n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < m; ++q) {
        int pix = pixels[q];
        pixel_spectrum(&c, pix % p->W, pix / p->W, 0, p->n_lambda, spec + q * p->n_lambda,
                       p->events ? p->events + q * p->n_lambda : NULL,
                       p->prec_bound ? p->prec_bound + q * p->n_lambda : NULL);
    }
    photon_map_free(&phm);
    spectra_free(&sp);
    return 0;
}

void orc_shadow(const orc_scene *s, int32_t use_bvh, int64_t m, const double *o, const int32_t *skip,
                double lambda_nm, double *T)
{
    orc_render_params p;
    memset(&p, 0, sizeof(p));
    p.n_lambda = 1;
    p.lambda_nm = &lambda_nm;
    spectra sp;
    spectra_make(s, &p, &sp);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i)
        T[i] = shadow_T(s, &sp, use_bvh, o + 3 * i, skip ? skip[i] : -1, 0, lambda_nm, NULL, NULL, NULL, 0.0, NULL);
    spectra_free(&sp);
}
