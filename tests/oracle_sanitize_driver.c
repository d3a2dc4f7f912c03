/* Drives every entry point of the oracle on a small scene, for runs under
 * AddressSanitizer + UndefinedBehaviorSanitizer and ThreadSanitizer (the
 * OpenMP renders).  The scene: a Lambert floor, a clear pane whose glass and
 * thickness come from a distribution map, a bubbly pane, and a clear pane at
 * 45 degrees that throws the overhead sun onto a wall (so the photon map
 * stores photons).  Exits 0 when every call returns normally and its
 * results are finite; the sanitizers report and fail the run on any memory
 * error, undefined behaviour or data race. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/sdm_oracle.h"

#define NT 4     /* table wavelengths */
#define NL 3     /* render wavelengths */

static int finite_all(const double *a, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int quad(double *pos, int32_t *idx, int32_t *mat, int *nv, int *nt, const double c[4][3], int m)
{
    for (int q = 0; q < 4; ++q)
        for (int a = 0; a < 3; ++a) pos[3 * (*nv + q) + a] = c[q][a];
    const int v = *nv;
    const int32_t t[6] = {v, v + 1, v + 2, v, v + 2, v + 3};
    memcpy(idx + 3 * *nt, t, sizeof(t));
    mat[*nt] = m;
    mat[*nt + 1] = m;
    *nv += 4;
    *nt += 2;
    return v;
}

int main(void)
{
    int fails = 0;
    double lam_tab[NT] = {380, 520, 660, 780}, n1[NT] = {1.53, 1.52, 1.515, 1.51}, k1[NT] = {1e-7, 1e-7, 1e-7, 1e-7};
    double tint1[NT] = {0.3, 0.1, 0.2, 0.4}, n2[NT] = {1.62, 1.61, 1.60, 1.60}, tint2[NT] = {1.5, 0.2, 0.1, 0.8};
    double alb[NT] = {0.5, 0.6, 0.6, 0.5}, sunE[NT] = {1, 1.2, 1.1, 0.9}, sky[NT] = {0.3, 0.3, 0.2, 0.2};
    orc_material mats[5];
    memset(mats, 0, sizeof(mats));
    mats[0].type = ORC_LAMBERT;
    mats[0].albedo = alb;
    mats[1].type = ORC_GLASS;      /* mapped pane */
    mats[1].thick_mm = 3.0;
    mats[1].n = n1; mats[1].k = k1; mats[1].alpha_tint = tint1;
    mats[1].dist_map = 1;
    mats[2].type = ORC_GLASS;      /* map glass / mirror pane */
    mats[2].thick_mm = 3.0;
    mats[2].n = n2; mats[2].k = k1; mats[2].alpha_tint = tint2;
    mats[3].type = ORC_GLASS_BUBBLY;
    mats[3].thick_mm = 4.0;
    mats[3].bubble_density = 20.0;
    mats[3].bubble_rmin_um = 10.0; mats[3].bubble_rmax_um = 200.0;
    mats[3].n = n1; mats[3].k = k1; mats[3].alpha_tint = tint1;
    mats[4] = mats[2];             /* plain clear glass */
    mats[4].n = n1; mats[4].alpha_tint = tint1;

    double pos[3 * 20], uv[2 * 20];
    int32_t idx[3 * 10], mat[10];
    int nv = 0, nt = 0;
    const double floor_[4][3] = {{-2, -2, 0}, {2, -2, 0}, {2, 2, 0}, {-2, 2, 0}};
    const double wall[4][3] = {{2, -2, 0}, {2, 2, 0}, {2, 2, 3}, {2, -2, 3}};
    const double pane[4][3] = {{-1.5, -1.5, 1}, {-0.5, -1.5, 1}, {-0.5, -0.5, 1}, {-1.5, -0.5, 1}};
    const double bub[4][3] = {{-1.5, 0.5, 1.2}, {-0.5, 0.5, 1.2}, {-0.5, 1.5, 1.2}, {-1.5, 1.5, 1.2}};
    const double a = 0.5 / sqrt(2.0);
    const double mirror[4][3] = {{0.8 - a, -0.5, 1 + a}, {0.8 + a, -0.5, 1 - a}, {0.8 + a, 0.5, 1 - a},
                                 {0.8 - a, 0.5, 1 + a}};
    memset(uv, 0, sizeof(uv));
    quad(pos, idx, mat, &nv, &nt, floor_, 0);
    quad(pos, idx, mat, &nv, &nt, wall, 0);
    const int vp = quad(pos, idx, mat, &nv, &nt, pane, 1);
    quad(pos, idx, mat, &nv, &nt, bub, 3);
    quad(pos, idx, mat, &nv, &nt, mirror, 4);
    const double puv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    for (int q = 0; q < 4; ++q) {
        uv[2 * (vp + q)] = puv[q][0];
        uv[2 * (vp + q) + 1] = puv[q][1];
    }
    int32_t texmat[6] = {2, 4, 2, 4, 2, 4};
    double texd[6] = {2.0, 3.0, 4.0, 5.0, 3.5, 2.5};
    orc_dist_map dm = {3, 2, texmat, texd};
    double vthick[20];
    for (int v = 0; v < nv; ++v) vthick[v] = 2.5 + 0.1 * v;

    orc_scene_desc d;
    memset(&d, 0, sizeof(d));
    d.nv = nv; d.pos = pos; d.vthick_mm = vthick; d.nt = nt; d.idx = idx; d.mat = mat;
    d.n_mat = 5; d.mats = mats; d.n_tab = NT; d.tab_lambda_nm = lam_tab;
    d.sun_dir[0] = 0.1; d.sun_dir[1] = 0.05; d.sun_dir[2] = sqrt(1 - 0.0125);
    d.sun_E = sunE; d.sky_L = sky; d.uv = uv; d.n_maps = 1; d.maps = &dm;
    orc_scene *s = orc_scene_create(&d);
    if (!s) {
        fprintf(stderr, "scene rejected\n");
        return 1;
    }

    double lam[NL] = {450, 550, 650}, cmf[3 * NL] = {0.3, 0.04, 1.7, 0.43, 0.99, 0.01, 0.28, 0.11, 0.0};
    orc_render_params p;
    memset(&p, 0, sizeof(p));
    p.W = 12; p.H = 10; p.spp = 3; p.max_depth = 5;
    p.eye[0] = 0.5; p.eye[1] = -1.8; p.eye[2] = 1.6;
    p.target[0] = 1.0; p.target[1] = 0.2; p.target[2] = 0.6;
    p.up[2] = 1.0; p.vfov_deg = 70.0; p.ortho_height = 1.0;
    p.seed = 7; p.job_id = 1; p.n_lambda = NL; p.lambda_nm = lam; p.cmf_xyz = cmf;
    p.n_bands = 2; p.tile = 4; p.use_bvh = 1; p.n_threads = 4;
    p.prec_rel = 6e-8; p.prec_ceps = 1e-7; p.prec_eps = 6e-8;
    p.photons = 20000; p.photon_radius = 0.2;
    const long npix = (long)p.W * p.H;
    double *spec = calloc((size_t)npix * NL, sizeof(double)), *xyz = calloc((size_t)npix * 3, sizeof(double));
    double *bound = calloc((size_t)npix * NL, sizeof(double));
    uint64_t *ev = calloc((size_t)npix * NL, sizeof(uint64_t));
    p.events = ev;
    p.prec_bound = bound;
    if (orc_render(s, &p, spec, xyz) != 0 || !finite_all(spec, npix * NL) || !finite_all(xyz, npix * 3)) {
        fprintf(stderr, "render failed\n");
        ++fails;
    }
    /* brute-force intersection, half the items, orthographic */
    p.use_bvh = 0; p.item_begin = 3; p.max_items = 5; p.projection = 1; p.photons = 0;
    p.events = NULL; p.prec_bound = NULL;
    if (orc_render(s, &p, spec, xyz) != 0) ++fails;
    p.projection = 0; p.item_begin = 0; p.max_items = 0; p.use_bvh = 1;
    int32_t pix[4] = {0, 17, 55, (int32_t)npix - 1};
    double pspec[4 * NL];
    if (orc_render_pixels(s, &p, 4, pix, pspec) != 0 || !finite_all(pspec, 4 * NL)) ++fails;
    p.photons = 20000;
    const int64_t nph = orc_photon_map(s, &p, NULL);
    if (nph <= 0) {
        fprintf(stderr, "no photons stored\n");
        ++fails;
    } else {
        double *ph = malloc((size_t)nph * 8 * sizeof(double));
        orc_photon_map(s, &p, ph);
        if (!finite_all(ph, nph * 8)) ++fails;
        free(ph);
    }
    /* rays, both walks */
    double o[6] = {0.1, -1.0, 2.5, -1.0, 1.0, 0.5}, dir[6] = {0.0, 0.3, -1.0, 0.2, -0.1, 1.0};
    const int32_t skip[2] = {-1, 3};
    for (int bvh = 0; bvh < 2; ++bvh) {
        double t[2], u[2], v[2], T[2];
        int32_t tri[2];
        orc_intersect(s, bvh, 2, o, dir, skip, t, tri, u, v);
        orc_shadow(s, bvh, 2, o, skip, 550.0, T);
        if (!finite_all(T, 2)) ++fails;
    }
    int32_t mt;
    double th;
    orc_pane_at(s, 4, 0.3, 0.2, &mt, &th);
    orc_scene_destroy(s);

    /* slab optics and the bubbly walk */
    double cos_i[2] = {0.9, 0.3}, lm[2] = {500, 620}, dmm[2] = {3.0, 4.5}, rho[2] = {5.0, 30.0};
    double nn[2] = {1.52, 1.55}, kk[2] = {1e-7, 2e-7}, tt[2] = {0.2, 0.5}, R[2], T2[2], A[2], W[2];
    orc_slab_mc(2, cos_i, lm, dmm, rho, 10.0, 200.0, nn, kk, tt, NULL, 3, 0, 256, R, T2, A, W);
    if (!finite_all(R, 2) || !finite_all(T2, 2)) ++fails;
    orc_walk_stream ws = {11, 3, 4, 0, 2, 1};
    orc_walk_out wo;
    orc_bubbly_walk(&ws, 0.7, 4.0, orc_bubble_sigma(25.0, 10.0, 200.0), 1.52, 1, &wo);

    /* the surrogate network */
    const int32_t npanes = 3;
    const int64_t P = orc_mlp_nparams(npanes);
    double *prm = malloc((size_t)P * sizeof(double)), *grad = malloc((size_t)P * sizeof(double));
    for (int64_t i = 0; i < P; ++i) prm[i] = 0.05 * sin(0.7 * (double)i);
    double tup[3 * 4] = {0.8, 500, 3.0, 10.0, 0.4, 650, 4.0, 25.0, 0.95, 420, 2.2, 0.0};
    int32_t pn[3] = {0, 2, 1};
    double out[9], tgt[9] = {0.1, 0.8, 0.2, 0.05, 0.9, 0.1, 0.2, 0.6, 0.3};
    orc_mlp_forward(prm, npanes, 3, tup, pn, out);
    const double loss = orc_mlp_loss_grad(prm, npanes, 3, tup, pn, tgt, grad);
    orc_mlp_forward_bf16(prm, npanes, 3, tup, pn, out);
    double bo[3], bb[3];
    orc_mlp_bf16_bound(prm, tup, 0, 1e-6, 1e-6, bo, bb);
    if (!isfinite(loss) || !finite_all(grad, P) || !finite_all(out, 9)) ++fails;
    free(prm);
    free(grad);
    free(spec);
    free(xyz);
    free(bound);
    free(ev);
    if (fails) fprintf(stderr, "%d checks failed\n", fails);
    else printf("oracle driver: all calls ran (%lld photons stored)\n", (long long)nph);
    return fails ? 1 : 0;
}
