/*
 * sdm_oracle.h -- plain FP64 CPU oracle of the spectral path tracer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * What it computes (paper: "Spectral Domain Decomposition Method for Natural
 * Lighting and Medieval Glass Rendering"):
 *   - inverse ray tracing from each pixel, closest hit, shadow rays toward the
 *     light, secondary rays by reflection/refraction, stop after a fixed
 *     number of bounces or below an energy threshold (Sec. 3.1);
 *   - the light sum of eq. (3) for the directional sun, the uniform sky as
 *     the escape radiance;
 *   - glass described by optical constants n + ik (eq. (1)) with thickness
 *     maps (Sec. 6);
 *   - each wavelength of the 81-sample grid handled on its own (Sec. 4), each
 *     pixel on its own (Sec. 4, Sec. 5), so any split into spectral bands and
 *     pixel tiles gives the same image.
 * Every other convention is a reading stated next to the code that uses it.
 */
#ifndef SDM_ORACLE_H
#define SDM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LAMBERT = 0, ORC_GLASS = 1, ORC_GLASS_BUBBLY = 2 };
/* How a path vertex on a bubbly pane is evaluated: the exact walk, the
 * surrogate network, or the network unless the error table flags the cell. */
enum { ORC_BTDF_EXACT = 0, ORC_BTDF_SURROGATE = 1, ORC_BTDF_FALLBACK = 2 };
/* Error-table cells: cos(theta) in [0, 1], thickness in [2, 5] mm, bubble
 * density in [0, 34] per mm^3, each split evenly (values outside clamp). */
#define ORC_ERR_D_LO 2.0
#define ORC_ERR_D_HI 5.0
#define ORC_ERR_RHO_HI 34.0

typedef struct {
    int32_t type;
    double thick_mm;          /* pane thickness when there is no per-vertex map */
    double bubble_density;    /* bubbles per mm^3 (bubbly glass) */
    double bubble_rmin_um, bubble_rmax_um;
    int32_t pane_id;
    const double *albedo;     /* [n_tab] or NULL */
    const double *n;          /* [n_tab] or NULL */
    const double *k;          /* [n_tab] or NULL */
    const double *alpha_tint; /* [n_tab] mm^-1 or NULL */
    int32_t dist_map;         /* clear glass: 1 + index of its distribution map, 0 none */
} orc_material;

/* Distribution map (Sec. 6): W x H texels over texture space [0, 1]^2, row 0
 * at t = 0.  At texture coordinates (s, t) a pane takes the material of
 * texel (clamp(floor(s W), 0, W - 1), clamp(floor(t H), 0, H - 1)) and, with
 * a thickness table, the bilinear interpolation of the texel thicknesses with
 * texel centres at ((x + 0.5) / W, (y + 0.5) / H), clamped at the edges. */
typedef struct {
    int32_t W, H;
    const int32_t *material;  /* [W*H] clear-glass material indices */
    const double *thick_mm;   /* [W*H] or NULL (the triangle's own thickness) */
} orc_dist_map;

typedef struct {
    int32_t nv;
    const double *pos;        /* [nv*3] metres */
    const double *vthick_mm;  /* [nv] or NULL */
    int32_t nt;
    const int32_t *idx;       /* [nt*3] */
    const int32_t *mat;       /* [nt] */
    int32_t n_mat;
    const orc_material *mats;
    int32_t n_tab;
    const double *tab_lambda_nm; /* [n_tab], increasing */
    double sun_dir[3];        /* unit vector toward the sun */
    const double *sun_E;      /* [n_tab] */
    const double *sky_L;      /* [n_tab] */
    const double *uv;         /* [nv*2] texture coordinates, or NULL */
    int32_t n_maps;
    const orc_dist_map *maps; /* [n_maps] */
} orc_scene_desc;

typedef struct {
    int32_t W, H, spp, max_depth;
    int32_t projection;       /* 0 pinhole, 1 orthographic */
    double eye[3], target[3], up[3];
    double vfov_deg, ortho_height;
    uint64_t seed;
    uint32_t job_id;
    int32_t n_lambda;
    const double *lambda_nm;  /* [n_lambda] */
    const double *cmf_xyz;    /* [n_lambda*3] */
    int32_t n_bands;          /* spectral subdomains (result is independent) */
    int32_t tile;             /* pixel-tile side of the work items */
    double beta_threshold;    /* energy threshold of Sec. 3.1 (0 = off) */
    int32_t use_bvh;          /* 1: BVH, 0: brute force */
    int32_t n_threads;        /* 0 = OpenMP default */
    /* bubbly panes */
    int32_t btdf_mode;        /* ORC_BTDF_* */
    int32_t mlp_n_panes;      /* embedding rows of the network */
    int32_t mlp_bf16;         /* 1: network with BF16 operands */
    int32_t err_dims[3];      /* cells along cos, thickness, density */
    const double *mlp_params; /* network parameters (ORC_BTDF_SURROGATE / _FALLBACK) */
    const double *err_table;  /* [mlp_n_panes][err_dims[0]][err_dims[1]][err_dims[2]] */
    double err_bound;         /* a cell above this uses the exact walk */
    /* Work items (pixel tile x band, tile rows top to bottom, tiles left to
     * right, bands in order): orc_render renders items [item_begin,
     * item_begin + max_items) only (max_items 0: every item from
     * item_begin) and leaves the other entries of spec untouched. */
    int64_t item_begin, max_items;
    /* Event signatures or NULL: [H*W*n_lambda] for orc_render, [m*n_lambda]
     * for orc_render_pixels.  Entry (pixel, lambda) = sum modulo 2^64, over
     * the pixel's paths at that wavelength, of a hash of each closest hit
     * (vertex, sample, triangle or none) and each shadow-ray result (vertex,
     * occluded or the set of panes crossed), counted while the path's
     * weight is nonzero; see event_hash in sdm_oracle.c. */
    uint64_t *events;
    /* Single-precision error bound or NULL (same layout as events): per
     * spectral pixel, a first-order bound on how far an evaluation of the
     * same paths (same decisions) in single precision can land from this
     * one.  Each contribution to the pixel adds |contribution| times the
     * relative error bound of its factors: prec_rel per factor, prec_ceps /
     * cos for the cosine of a light sum, and for each glass factor (a glass hit on the path, or a pane its shadow ray
     * crosses) prec_ceps / c + alpha |grad d| h / cos_t, where c is the
     * incidence cosine, cos_t the refracted one, alpha = 4 pi k / lambda +
     * alpha_tint (per mm), |grad d| the thickness gradient across the pane
     * triangle (mm per m) and h the error bound of the hit within the pane.
     * Hit errors follow the path: a hit reached from an origin with error e
     * over a distance t at incidence cosine c has error (e + prec_eps t) / c
     * + prec_eps |x| (the ray's offset moves the hit within the surface by
     * that over c; the hit is then rounded); a camera origin has prec_eps
     * |x|.  prec_eps bounds the relative rounding of positions and
     * directions, prec_ceps the error of a cosine formed from them. */
    double *prec_bound;
    double prec_rel, prec_ceps, prec_eps;
    /* Caustic photon map (photon mapping, Sec. 3.2; 0 photons: off): photons
     * shot from the sun and stored where a pane has turned them; every
     * Lambert vertex adds rho / pi times the stored power of its wavelength
     * within photon_radius (metres) divided by pi r^2 (see orc_photon_map). */
    int64_t photons;
    double photon_radius;
} orc_render_params;

typedef struct orc_scene orc_scene;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out);
double orc_u01(uint32_t x);

/* Interface Fresnel reflectance, air -> n + ik, per polarisation. */
void orc_fresnel(double cos_i, double n, double k, double *Rs, double *Rp);
/* The caustic photon map of a render (test instrument view of the first
 * pass): the photons stored, as rows (x, y, z, nx, ny, nz, power, j);
 * returns the count, or -1.  out may be NULL to count only. */
int64_t orc_photon_map(const orc_scene *s, const orc_render_params *p, double *out);
/* Material and thickness of the pane of triangle t at barycentric (u, v):
 * with a distribution map, its texel's material and thickness (see
 * orc_dist_map); otherwise the triangle's material and thickness. */
void orc_pane_at(const orc_scene *s, int32_t t, double u, double v, int32_t *material, double *thick_mm);
/* Thin slab: incoherent multiple reflection with Beer-Lambert attenuation. */
void orc_slab(double cos_i, double lambda_nm, double d_mm, double n, double k,
              double alpha_tint, double *R, double *T);
void orc_slab_batch(int64_t m, const double *cos_i, const double *lambda_nm,
                    const double *d_mm, const double *n, const double *k,
                    const double *alpha_tint, double *R, double *T);
/* Refraction angle used for the path length (real Snell). */
double orc_snell_cos_t(double cos_i, double n);

orc_scene *orc_scene_create(const orc_scene_desc *d);
void orc_scene_destroy(orc_scene *s);
double orc_scene_teps(const orc_scene *s);
int32_t orc_bvh_depth(const orc_scene *s);

/* Closest hit of m rays; tri = -1 on a miss.  skip[i] is a triangle to ignore. */
void orc_intersect(const orc_scene *s, int32_t use_bvh, int64_t m, const double *o,
                   const double *dir, const int32_t *skip, double *t, int32_t *tri,
                   double *u, double *v);
/* Sun transmittance from m points (0 if an opaque triangle is in the way). */
void orc_shadow(const orc_scene *s, int32_t use_bvh, int64_t m, const double *o,
                const int32_t *skip, double lambda_nm, double *T);

/* Whole image: spec[H*W*n_lambda] (lambda fastest) and xyz[H*W*3]. */
int orc_render(const orc_scene *s, const orc_render_params *p, double *spec, double *xyz);
/* Selected pixels only: spec[m*n_lambda]. */
int orc_render_pixels(const orc_scene *s, const orc_render_params *p, int64_t m,
                      const int32_t *pixels, double *spec);
/* Camera ray for image point (i + u0, j + u1) (exposed for the pin tests). */
void orc_camera_ray(const orc_render_params *p, int32_t i, int32_t j, double u0, double u1,
                    double o[3], double d[3]);
/* Cosine-weighted direction about unit n from (u1, u2) (exposed for tests). */
void orc_cosine_dir(const double n[3], double u1, double u2, double d[3]);
/* Transmitted direction of the surrogate: d tilted by a 2-D Gaussian of
 * standard deviation w (radians, per tangent axis) from (u1, u2). */
void orc_lobe_dir(const double d[3], double w, double u1, double u2, double out[3]);
/* The transmitted direction the surrogate form takes at a pane of normal ng:
 * orc_lobe_dir, mirrored across the pane's plane when it points back to the
 * side the ray came from. */
void orc_lobe_transmit(const double d[3], const double ng[3], double w, double u1, double u2, double out[3]);
/* Direction a (slab frame of orc_bubbly_walk) in world space for a ray d
 * hitting a face of geometric normal ng. */
void orc_slab_to_world(const double d[3], const double ng[3], const double a[3], double out[3]);

/* Spectral image -> XYZ with trapezoid weights in nm. */
void orc_spec_to_xyz(int64_t npix, int32_t n_lambda, const double *lambda_nm,
                     const double *cmf_xyz, const double *spec, double *xyz);

/* Bubbly slab Monte Carlo (reading; see slab_mc.c): m tuples of n_photons
 * photons; outputs R, T, A (absorbed) and the transmitted-lobe width.
 * n_ref: the real index used inside the slab (NULL = n). */
void orc_slab_mc(int64_t m, const double *cos_i, const double *lambda_nm, const double *d_mm,
                 const double *rho_b, double rmin_um, double rmax_um, const double *n, const double *k,
                 const double *alpha_tint, const double *n_ref, uint64_t seed, uint32_t tuple0,
                 int32_t n_photons, double *R, double *T, double *A, double *w_lobe);

/* Draw stream of one walk: render = 0 -> dataset counters (c0 = tuple,
 * c1 = photon); render = 1 -> (c0 = pixel, c1 = sample, vertex, c3 = job). */
typedef struct {
    uint64_t seed;
    uint32_t c0, c1, c3, vertex;
    int32_t render;
} orc_walk_stream;

typedef struct {
    int32_t kind;   /* 0 absorbed (event cap), 1 out through the entry face, 2 through the far face */
    double dir[3];  /* direction in air, slab frame (x in the plane of incidence, z into the slab) */
    double L;       /* geometric length travelled in glass (mm) */
    int32_t n_events; /* free flights taken (bubbles met and faces reached) */
    int32_t bubbles;  /* bubbles met (0: the light left unscattered) */
} orc_walk_out;

/* The four uniforms of draw (event, sub) of a walk stream. */
void orc_walk_draw(const orc_walk_stream *st, uint32_t event, uint32_t sub, double u[4]);
void orc_bubbly_walk(const orc_walk_stream *st, double cos_i, double d_mm, double sigma, double n_ref,
                     int pol, orc_walk_out *out);
/* Extinction of the bubbles, rho_b pi <r^2> with r ~ U(rmin, rmax) (per mm). */
double orc_bubble_sigma(double rho_b, double rmin_um, double rmax_um);
double orc_fresnel_real(double n1, double n2, double c, int pol);
void orc_bubble_dir(const double dir[3], const double e_perp[3], double sin_i, double n, int p, double out[3]);

/* Surrogate network (reading; see mlp.c). */
int64_t orc_mlp_nparams(int32_t n_panes);
void orc_mlp_forward(const double *params, int32_t n_panes, int64_t m, const double *tuples,
                     const int32_t *panes, double *out);
double orc_mlp_loss_grad(const double *params, int32_t n_panes, int64_t m, const double *tuples,
                         const int32_t *panes, const double *target, double *grad);
/* The same network with BF16 operands (matrix-core arithmetic). */
/* Test instrument: one tuple's BF16-operand outputs (R, T, w) and a bound on
 * their distance from an evaluation with FP32 sums whose cos and thickness
 * inputs are off by up to e_cos and e_d (see mlp.c). */
void orc_mlp_bf16_bound(const double *params, const double *tup, int32_t pane, double e_cos, double e_d,
                        double out[3], double bound[3]);
void orc_mlp_forward_bf16(const double *params, int32_t n_panes, int64_t m, const double *tuples,
                          const int32_t *panes, double *out);
double orc_bf16(double x);

#ifdef __cplusplus
}
#endif
#endif
