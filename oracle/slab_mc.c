/*
 * slab_mc.c -- FP64 Monte Carlo of a glass slab holding spherical air
 * bubbles (test infrastructure, part of the CPU oracle).
 *
 * The paper names the phenomenon only: air micro-particles inside medieval
 * glass scatter light in volume (Sec. 1), and light scattering is named as
 * the next material feature (Sec. 6).  The walk below is a reading:
 *   - slab of thickness d with optical constants n + ik (eq. (1)); the entry
 *     interface uses the complex index at the wavelength, per polarisation;
 *   - inside, directions and decisions (faces, bubbles) use one real index
 *     n_ref per pane (its index at 560 nm in a render), so the walk does not
 *     depend on the wavelength; bubble optics are only weakly dispersive;
 *   - Beer-Lambert weight exp(-alpha L) over the length L travelled in glass,
 *     alpha = 4 pi k / lambda + alpha_tint;
 *   - bubbles: Poisson centres of density rho_b, radii uniform in
 *     [rmin, rmax]; extinction sigma = rho_b pi <r^2>; a bubble acts at the
 *     collision point (its size, <= 0.2 mm, is neglected for the position)
 *     with exact sphere geometric optics for the direction: impact ratio
 *     b / r = sqrt(u), glass -> air Fresnel or total reflection at the first
 *     surface, else p internal reflections (air -> glass Fresnel each time)
 *     and a total deviation 2 (i - r) + p (pi - 2 r) away from the centre;
 *     the polarisation label is drawn afresh after each bubble;
 *   - a photon leaving the top face counts toward R, the bottom face toward
 *     T; the lobe width is the weighted RMS angle between transmitted and
 *     incident directions, divided by sqrt(2).
 * Random numbers: Philox4x32-10 with the 64-bit seed as key and the counter
 * of orc_walk_draw().
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "sdm_oracle.h"

#define PI 3.14159265358979323846
#define MC_MAX_EVENTS 10000
#define MC_MAX_INTERNAL 64

static void mc_draw(uint64_t seed, uint32_t tuple, uint32_t photon, uint32_t event, uint32_t sub, double u[4])
{
    uint32_t ctr[4] = {tuple, photon, event, 0x5EB10000u | sub};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = orc_u01(x[i]);
}

/* Fresnel reflectance of a real interface n1 -> n2 at incidence cosine c for
 * polarisation pol (0 = s, 1 = p); 1 beyond the critical angle. */
double orc_fresnel_real(double n1, double n2, double c, int pol)
{
    if (c > 1.0) c = 1.0;
    double s2 = 1.0 - c * c;
    double st2 = (n1 / n2) * (n1 / n2) * s2;
    if (st2 >= 1.0) return 1.0;
    double ct = sqrt(1.0 - st2);
    double r = pol == 0 ? (n1 * c - n2 * ct) / (n1 * c + n2 * ct) : (n2 * c - n1 * ct) / (n2 * c + n1 * ct);
    return r * r;
}

static void cross(const double *a, const double *b, double *r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static void unit(double *a)
{
    double l = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    if (l > 0) { a[0] /= l; a[1] /= l; a[2] /= l; }
}

/* Direction after a bubble, given its outcome.  dir: unit direction in
 * glass; e_perp: unit vector from the bubble centre toward the ray's impact
 * point (perpendicular to dir); sin_i: impact ratio b / r; p: number of
 * internal reflections, or -1 for a reflection at the outer surface. */
void orc_bubble_dir(const double dir[3], const double e_perp[3], double sin_i, double n, int p, double out[3])
{
    double cos_i = sqrt(fmax(0.0, 1.0 - sin_i * sin_i));
    if (p < 0) {
        /* outward normal at the hit point: -cos_i dir + sin_i e_perp */
        double nh[3], dn = 0.0;
        for (int a = 0; a < 3; ++a) nh[a] = -cos_i * dir[a] + sin_i * e_perp[a];
        for (int a = 0; a < 3; ++a) dn += dir[a] * nh[a];
        for (int a = 0; a < 3; ++a) out[a] = dir[a] - 2.0 * dn * nh[a];
        return;
    }
    double ri = asin(fmin(sin_i, 1.0)), rr = asin(fmin(n * sin_i, 1.0));
    double D = 2.0 * (ri - rr) + p * (PI - 2.0 * rr);
    for (int a = 0; a < 3; ++a) out[a] = cos(D) * dir[a] - sin(D) * e_perp[a];
}

/* Tangent basis about unit n from the fixed axis h = (1, 2, 3) / sqrt(14). */
static void basis(const double *n, double *t1, double *t2)
{
    const double h[3] = {0.2672612419124244, 0.5345224838248488, 0.8017837257372732};
    cross(h, n, t1);
    unit(t1);
    cross(n, t1, t2);
}

/* Counter of the walk's draws.  Tables of the slab (dataset): (tuple,
 * photon, event, 0x5EB10000 | sub).  Inside a render, at path vertex v of
 * (pixel, sample, job): (pixel, sample, 2^31 | v << 23 | event << 5 | sub,
 * job); bit 31 keeps these apart from the per-vertex draws, whose third word
 * is below 2^24. */
void orc_walk_draw(const orc_walk_stream *st, uint32_t event, uint32_t sub, double u[4])
{
    if (!st->render) {
        mc_draw(st->seed, st->c0, st->c1, event, sub, u);
        return;
    }
    uint32_t ctr[4] = {st->c0, st->c1, 0x80000000u | (st->vertex << 23) | (event << 5) | sub, st->c3};
    uint32_t key[2] = {(uint32_t)st->seed, (uint32_t)(st->seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = orc_u01(x[i]);
}

/* The walk inside the slab after the photon has entered (reading): every
 * direction and every internal decision (face reflections, bubble surfaces)
 * uses the pane's real index n_ref; only the entry interface and the
 * absorption depend on the wavelength.  So the walk is the same for every
 * wavelength that enters, and its absorption weight is exp(-alpha L) with L
 * the geometric length travelled in glass.  pol: polarisation label drawn at
 * entry.  Output direction in air, slab frame: x in the plane of incidence,
 * z into the slab; kind 1 = left through the entry face, 2 = through the far
 * face, 0 = event cap reached (absorbed). */
void orc_bubbly_walk(const orc_walk_stream *st, double cos_i, double d, double sigma, double n_ref, int pol,
                     orc_walk_out *out)
{
    double u[4], v[4];
    double sin_i = sqrt(fmax(0.0, 1.0 - cos_i * cos_i));
    double st_ = sin_i / n_ref;
    double dir[3] = {st_, 0.0, sqrt(fmax(0.0, 1.0 - st_ * st_))};
    double z = 0.0, L = 0.0;
    out->kind = 0;
    out->dir[0] = out->dir[1] = out->dir[2] = 0.0;
    out->n_events = 0;
    out->bubbles = 0;
    for (uint32_t e = 1; e <= MC_MAX_EVENTS; ++e) {
        out->n_events = (int32_t)e;
        orc_walk_draw(st, e, 0, u);
        double sb = dir[2] > 0.0 ? (d - z) / dir[2] : (dir[2] < 0.0 ? -z / dir[2] : INFINITY);
        double l = sigma > 0.0 ? -log1p(-u[0]) / sigma : INFINITY;
        if (l >= sb) {
            L += sb;
            int bottom = dir[2] > 0.0;
            z = bottom ? d : 0.0;
            if (u[1] < orc_fresnel_real(n_ref, 1.0, fabs(dir[2]), pol)) {
                dir[2] = -dir[2];
                continue;
            }
            double tx = n_ref * dir[0], ty = n_ref * dir[1];
            double tz = sqrt(fmax(0.0, 1.0 - tx * tx - ty * ty));
            out->kind = bottom ? 2 : 1;
            out->dir[0] = tx;
            out->dir[1] = ty;
            out->dir[2] = bottom ? tz : -tz;
            out->L = L;
            return;
        }
        L += l;
        z += l * dir[2];
        ++out->bubbles;
        /* bubble: impact ratio sqrt(u2), azimuth 2 pi u3 about dir; the
         * polarisation label relative to the bubble is drawn afresh */
        double t1[3], t2[3], ep[3];
        basis(dir, t1, t2);
        double phi = 2.0 * PI * u[3];
        for (int a = 0; a < 3; ++a) ep[a] = cos(phi) * t1[a] + sin(phi) * t2[a];
        uint32_t sub = 1;
        orc_walk_draw(st, e, sub, v);
        pol = v[1] < 0.5 ? 0 : 1;
        double sin_b = sqrt(u[2]), cos_b = sqrt(1.0 - u[2]);
        int p;
        if (v[0] < orc_fresnel_real(n_ref, 1.0, cos_b, pol)) {
            p = -1;
        } else {
            double sr = n_ref * sin_b;
            double R2 = orc_fresnel_real(1.0, n_ref, sqrt(fmax(0.0, 1.0 - sr * sr)), pol);
            int q = 2;
            p = 0;
            while (p < MC_MAX_INTERNAL) {
                if (q == 4) {
                    orc_walk_draw(st, e, ++sub, v);
                    q = 0;
                }
                if (v[q++] < R2) ++p;
                else break;
            }
        }
        double ndir[3];
        orc_bubble_dir(dir, ep, sin_b, n_ref, p, ndir);
        for (int a = 0; a < 3; ++a) dir[a] = ndir[a];
        unit(dir);
    }
    out->L = L;   /* event cap reached: absorbed */
}

typedef struct {
    double R, T, A, dev2;
} mc_acc;

/* One photon of a dataset tuple: entry interface with the complex index at
 * lambda (eq. (1)), polarisation label, then the walk. */
static void mc_photon(double cos_i, double lambda_nm, double d, double sigma, double n, double k, double tint,
                      double n_ref, uint64_t seed, uint32_t tuple, uint32_t ph, mc_acc *acc)
{
    double u[4];
    double sin_i = sqrt(fmax(0.0, 1.0 - cos_i * cos_i));
    const double inc[3] = {sin_i, 0.0, cos_i};
    orc_walk_stream st = {seed, tuple, ph, 0, 0, 0};
    orc_walk_draw(&st, 0, 0, u);
    int pol = u[1] < 0.5 ? 0 : 1;
    double Rs, Rp;
    orc_fresnel(cos_i, n, k, &Rs, &Rp);
    if (u[0] < (pol == 0 ? Rs : Rp)) {
        acc->R += 1.0;
        return;
    }
    orc_walk_out w;
    orc_bubbly_walk(&st, cos_i, d, sigma, n_ref, pol, &w);
    if (w.kind == 0) {
        acc->A += 1.0;
        return;
    }
    double alpha = 4.0 * PI * k / (lambda_nm * 1e-6) + tint;
    double wt = exp(-alpha * w.L);
    if (w.kind == 2) {
        acc->T += wt;
        double c = w.dir[0] * inc[0] + w.dir[1] * inc[1] + w.dir[2] * inc[2];
        double dev = acos(fmax(-1.0, fmin(1.0, c)));
        acc->dev2 += wt * dev * dev;
    } else {
        acc->R += wt;
    }
    acc->A += 1.0 - wt;
}

double orc_bubble_sigma(double rho_b, double rmin_um, double rmax_um)
{
    const double a = rmin_um * 1e-3, b = rmax_um * 1e-3;
    return rho_b * PI * ((a * a + a * b + b * b) / 3.0);
}

void orc_slab_mc(int64_t m, const double *cos_i, const double *lambda_nm, const double *d_mm,
                 const double *rho_b, double rmin_um, double rmax_um, const double *n, const double *k,
                 const double *alpha_tint, const double *n_ref, uint64_t seed, uint32_t tuple0, int32_t n_photons,
                 double *R, double *T, double *A, double *w_lobe)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < m; ++i) {
        mc_acc acc = {0, 0, 0, 0};
        double sigma = orc_bubble_sigma(rho_b[i], rmin_um, rmax_um);
        double nr = n_ref ? n_ref[i] : n[i];
        for (int32_t p = 0; p < n_photons; ++p)
            mc_photon(cos_i[i], lambda_nm[i], d_mm[i], sigma, n[i], k[i], alpha_tint[i], nr, seed,
                      tuple0 + (uint32_t)i, (uint32_t)p, &acc);
        R[i] = acc.R / n_photons;
        T[i] = acc.T / n_photons;
        if (A) A[i] = acc.A / n_photons;
        w_lobe[i] = acc.T > 0.0 ? sqrt(acc.dev2 / acc.T) / sqrt(2.0) : 0.0;
    }
}
