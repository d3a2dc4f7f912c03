/*
 * sdm.h -- C ABI of the MI355X spectral path tracer (libsdm.so).
 *
 * The library renders naturally lit scenes with glass panes, per pixel and
 * per wavelength, as in "Spectral Domain Decomposition Method for Natural
 * Lighting and Medieval Glass Rendering":
 *   - inverse ray tracing from the pixels, closest hit, a shadow ray to the
 *     light, reflected/refracted secondaries, stop after a fixed number of
 *     bounces or below an energy threshold (Sec. 3.1);
 *   - the light sum of eq. (3) over the directional sun, a uniform sky as the
 *     radiance of escaping rays;
 *   - glass panes described by optical constants n + ik (eq. (1)) with
 *     per-vertex thickness maps (Sec. 6), as thin slabs with Fresnel
 *     interfaces and Beer-Lambert absorption;
 *   - the spectral (wavelength-band) and ray-set (pixel-tile) sub-domains of
 *     Sec. 4 and Sec. 5 become work items of one GPU; the result does not
 *     depend on how they are cut;
 *   - spectral radiance is accumulated in FP64 and converted to CIE XYZ with
 *     a caller-supplied observer table.
 *
 * Conventions for every function:
 *   - returns SDM_OK (0) or a negative SDM_E_* code; sdm_last_error() then
 *     describes the failure.  Nothing is written to outputs on SDM_E_INVALID.
 *   - scene and parameter arrays are HOST pointers and are copied during the
 *     call (the caller may free them on return), unless stated otherwise.
 *   - output buffers are owned by the caller; their memory kind (host or
 *     device) is given per buffer.
 *   - work is enqueued on the caller's HIP stream (hip_stream, may be NULL for
 *     the null stream).  Device outputs are valid once that stream is
 *     synchronised; host outputs are valid on return.
 *   - a context is not thread-safe: use one context per host thread.  Scenes
 *     belong to the context that created them; destroy them before it.
 */
#ifndef SDM_H
#define SDM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDM_OK 0
#define SDM_E_INVALID (-1)     /* bad argument (null pointer, size, index)   */
#define SDM_E_NOMEM (-2)       /* device or host allocation failed            */
#define SDM_E_DEVICE (-3)      /* HIP error or a device-side error flag       */
#define SDM_E_UNSUPPORTED (-4) /* valid request this build does not handle    */
#define SDM_E_ABORTED (-5)     /* the render's item budget ran out; resumable  */

enum { SDM_LAMBERT = 0, SDM_GLASS = 1, SDM_GLASS_BUBBLY = 2 };
enum { SDM_MEM_HOST = 0, SDM_MEM_DEVICE = 1 };
enum { SDM_PREC_FP32 = 0, SDM_PREC_FP64 = 1 };
enum { SDM_PINHOLE = 0, SDM_ORTHO = 1 };
/* How shadow rays (all along the scene's sun direction) find what they cross:
 * a grid over the triangles projected along the sun where it is compact, else
 * the BVH; or always the BVH.  Both report the same crossings (the same
 * triangle test decides). */
enum { SDM_SHADOW_AUTO = 0, SDM_SHADOW_BVH = 1 };
/* Evaluation of path vertices on bubbly panes (SDM_GLASS_BUBBLY). */
enum { SDM_BTDF_EXACT = 0, SDM_BTDF_SURROGATE = 1, SDM_BTDF_FALLBACK = 2 };

/* Interface hand-off of geometric sub-domains (sdm_scene_desc). */
enum { SDM_HANDOFF_QUEUE = 0, SDM_HANDOFF_MARCH = 1 };

/* Largest number of wavelengths one spectral band (sub-domain) may hold. */
#define SDM_MAX_BAND 128

typedef struct sdm_context sdm_context;
typedef struct sdm_scene sdm_scene;
typedef struct sdm_mlp sdm_mlp;

/* Material.  Tables are host arrays sampled at the scene's tab_lambda_nm and
 * linearly interpolated to the render wavelengths (held constant beyond the
 * table ends).  Lambert needs albedo; glass needs n and k (eq. (1));
 * alpha_tint (mm^-1, extra absorption) may be NULL for zero. */
typedef struct {
    int32_t type;               /* SDM_LAMBERT, SDM_GLASS or SDM_GLASS_BUBBLY  */
    const float *albedo;        /* [n_tab] or NULL                             */
    const float *n;             /* [n_tab] real index, >= 1                    */
    const float *k;             /* [n_tab] absorption index, >= 0              */
    const float *alpha_tint;    /* [n_tab] mm^-1, or NULL                      */
    float thick_mm;             /* pane thickness when vthick_mm is NULL        */
    float bubble_density_mm3;   /* bubbly glass: air bubbles per mm^3, >= 0     */
    float bubble_rmin_um, bubble_rmax_um;   /* radius range (micrometres)      */
    int32_t pane_id;            /* bubbly glass: the network's pane type       */
    /* Clear glass only: 0, or k > 0 to take the optical constants and the
     * thickness at a hit from the scene's distribution map k - 1 (Sec. 6:
     * distribution maps of optical constants and of thickness over the
     * geometry, looked up through the hit's texture coordinates, Sec. 3.1). */
    int32_t dist_map;
} sdm_material;

/* Distribution map (Sec. 6): a W x H grid of texels over texture space
 * [0, 1]^2, row 0 at t = 0, column 0 at s = 0.  A hit at barycentric (u, v)
 * of triangle (i0, i1, i2) has texture coordinates
 * (s, t) = (1 - u - v) uv[i0] + u uv[i1] + v uv[i2].
 * Optical constants: the material of texel (clamp(floor(s W), 0, W - 1),
 * clamp(floor(t H), 0, H - 1)) -- an index of a clear-glass material of the
 * scene, whose n, k and alpha_tint tables apply at that hit.
 * Thickness: NULL keeps the triangle's thickness (vthick_mm, else the
 * material's thick_mm); otherwise the bilinear interpolation of thick_mm
 * with texel centres at ((x + 0.5) / W, (y + 0.5) / H), clamped at the
 * edges.  Arrays are host memory, row-major, copied by sdm_scene_create. */
typedef struct {
    int32_t W, H;               /* texels, 1 .. 4096 each                     */
    const int32_t *material;    /* [W*H] clear-glass material indices          */
    const float *thick_mm;      /* [W*H] thickness (> 0), or NULL              */
} sdm_dist_map;

/* Scene.  Triangles are two-sided.  Units: metres, thickness in mm. */
typedef struct {
    int32_t nv;
    const float *pos;           /* [nv*3]                                      */
    const float *vthick_mm;     /* [nv] per-vertex pane thickness, or NULL      */
    int32_t nt;
    const int32_t *idx;         /* [nt*3] vertex indices in [0, nv)             */
    const int32_t *mat;         /* [nt] material indices in [0, n_mat)          */
    int32_t n_mat;
    const sdm_material *mats;   /* [n_mat]                                      */
    int32_t n_tab;
    const float *tab_lambda_nm; /* [n_tab], strictly increasing                 */
    float sun_dir[3];           /* unit vector toward the sun                   */
    const float *sun_E;         /* [n_tab] sun irradiance                       */
    const float *sky_L;         /* [n_tab] uniform sky radiance                 */
    int32_t shadow_walk;        /* SDM_SHADOW_AUTO or SDM_SHADOW_BVH            */
    const float *uv;            /* [nv*2] texture coordinates, or NULL (required
                                   when a material has a distribution map)     */
    int32_t n_maps;
    const sdm_dist_map *maps;   /* [n_maps]                                    */
    /* Geometric sub-domains (Sec. 5): the scene's bounds cut into a grid of
     * subdomains[0] x [1] x [2] cells (0 or 1 along an axis: no cut; at most
     * 64 along an axis, 4096 cells), each with its own BVH over the triangles
     * that overlap it.  Closest hits of a single render are then found cell
     * by cell along each ray, rays crossing an interface being handed to the
     * neighbouring cell with their state; the image is the same as without
     * the cut.  Batches (sdm_render_batch) do not take such scenes. */
    int32_t subdomains[3];
    /* How a ray crosses an interface: SDM_HANDOFF_QUEUE, it waits in the
     * neighbouring cell's queue for the next pass (passes per bounce: the
     * most cells a ray can cross); SDM_HANDOFF_MARCH, the thread that traced
     * it goes on in the neighbour. */
    int32_t subdomain_handoff;
} sdm_scene_desc;

typedef struct {
    float eye[3], target[3], up[3];
    float vfov_deg;             /* pinhole vertical field of view              */
    float ortho_height;         /* orthographic view height (metres)           */
    int32_t W, H;
    int32_t projection;         /* SDM_PINHOLE or SDM_ORTHO                    */
} sdm_camera;

typedef struct {
    sdm_camera camera;
    int32_t n_lambda;           /* render wavelengths                          */
    const float *lambda_nm;     /* [n_lambda] host                             */
    const float *cmf_xyz;       /* [n_lambda*3] host observer table            */
    int32_t spp;                /* samples per pixel (>= 1)                    */
    int32_t max_depth;          /* shaded vertices per path (>= 1)             */
    uint64_t seed;              /* Philox key                                  */
    uint32_t job_id;            /* fourth Philox counter word                  */
    int32_t n_bands;            /* spectral sub-domains (>= 1), even split     */
    const int32_t *band_edges;  /* [n_bands+1] host, or NULL for an even split */
    int32_t tile_w, tile_h;     /* pixel-tile work items (0 = library default) */
    float beta_threshold;       /* path-weight threshold (0 = off)             */
    int32_t precision;          /* SDM_PREC_FP32 (default) or SDM_PREC_FP64    */
    int64_t chunk_paths;        /* in-flight primary paths (0: tuned, else 2^23) */
    int32_t timing;             /* 1: time every kernel with HIP events        */
    /* Bubbly panes.  SDM_BTDF_EXACT: the photon walk of sdm_slab_mc at each
     * vertex (entry interface per wavelength with n + ik, walk inside at the
     * pane's index at 560 nm shared by every wavelength, weight
     * exp(-alpha L)).  SDM_BTDF_SURROGATE: the network's (R, T) per
     * wavelength, reflect with probability R / (R + T) else a Gaussian lobe
     * of the network's width at 560 nm, weight R + T.  SDM_BTDF_FALLBACK: the
     * surrogate, except where err_table[pane][c][t][r] > err_bound for the
     * vertex's cell (c: cos theta in [0, 1], t: thickness in [2, 5] mm, r:
     * density in [0, 34] per mm^3, err_dims cells each, clamped), which take
     * the exact walk.  Shadow rays through bubbly panes see the slab
     * transmittance with the bubbles' extinction added to the absorption. */
    int32_t btdf_mode;
    int32_t err_dims[3];        /* cells along cos, thickness, density          */
    const sdm_mlp *mlp;         /* network (surrogate modes), same context      */
    const float *err_table;     /* host [n_panes * err_dims product] (fallback) */
    float err_bound;
    int32_t graph;              /* 1: replay each chunk's kernel sequence as a
                                   HIP graph (ignored when timing = 1)         */
    /* Work-item budget.  The spectral and ray-set sub-domains are independent
     * (Sec. 4 and 5), so a render may run as several calls.  0: render every
     * (pixel tile x band) item.  n > 0: render at most n of the items not yet
     * done, in plan order (tile rows top to bottom, tiles left to right,
     * bands in order); when items remain, the outputs hold the items done so
     * far (zero elsewhere), the context keeps the partial state and the call
     * returns SDM_E_ABORTED: sdm_render_resume continues it and
     * sdm_render_checkpoint saves it.  Single renders only: sdm_render_batch
     * returns SDM_E_UNSUPPORTED for max_items > 0. */
    int64_t max_items;
    /* Caustic photon map (photon mapping, Sec. 3.2).  0: off.  n > 0: before
     * the render, n sun photons of one render wavelength each leave a square
     * across the sun's direction covering the scene's bounding sphere
     * (centred two radii toward the sun; its axes h x s and s x (h x s)
     * normalised, s the sun direction, h = (1, 2, 3) / sqrt(14)) and follow
     * the panes (clear glass: reflect with probability R / (R + T), weight
     * R + T; bubbly glass: the exact walk) for up to max_depth vertices; a
     * photon that a pane has turned (reflected or scattered by bubbles) is
     * stored where it first meets a Lambert surface, with power
     * E_sun(lambda) x square area x n_lambda / n.  Every Lambert vertex of
     * the render then adds g b_j rho_j / pi x sum Phi / (pi r^2) over the
     * stored photons of its wavelength j within photon_radius r (metres)
     * whose arrival side's normal is within 0.9 (cosine) of its own.  Single
     * renders only; not with max_items. */
    int64_t photons;
    float photon_radius;
    /* Resident blocks per compute unit of the persistent closest-hit and
     * shadow-walk passes: 0 takes the library's choice (what sdm_autotune
     * chose for this render shape, else the most that fit, four for
     * sun-grid walks); n > 0 is capped at the most that fit.  The image
     * does not depend on it. */
    int32_t trace_blocks_per_cu, shadow_blocks_per_cu;
} sdm_render_params;

/* Kernel classes reported in sdm_stats. */
enum { SDM_K_GENERATE = 0, SDM_K_TRACE = 1, SDM_K_SHADE = 2, SDM_K_SHADOW = 3,
       SDM_K_FINALIZE = 4, SDM_K_SHADOW_ACCUM = 5, SDM_K_SHADE_GLASS = 6, SDM_K_BUBBLY_EVAL = 7,
       SDM_K_SHADE_BUBBLY = 8, SDM_K_PHOTON = 9, SDM_K_CAUSTIC = 10, SDM_K_COUNT = 11 };

typedef struct {
    uint64_t spectral_samples;  /* W*H*spp*n_lambda                            */
    uint64_t paths;             /* primary rays: pixels x spp x bands          */
    uint64_t closest_segments;  /* closest-hit traversals                      */
    uint64_t shadow_segments;   /* shadow (any-hit) traversals                 */
    uint64_t forks;             /* paths split at glass by wavelength          */
    uint64_t chunks;            /* wavefront chunks                            */
    uint64_t nodes_visited[2];  /* [closest-hit, shadow]: wide BVH node fetches;
                                   for shadow rays of a scene with a sun grid,
                                   grid candidates examined instead          */
    uint64_t tris_tested[2];    /* ray-triangle tests [closest-hit, shadow]    */
    uint64_t bubbly_vertices;   /* path vertices shaded on bubbly panes         */
    uint64_t spectral_paths;    /* closest-hit segments whose wavelengths carry
                                   different weights (per-wavelength factors)  */
    uint64_t spectral_records;  /* shadow records with per-wavelength factors   */
    uint64_t glass_vertices[2]; /* glass vertices shaded [all, those arriving
                                   with per-wavelength factors]               */
    double ms_render;          /* wall time of the render on the stream       */
    double kernel_ms[SDM_K_COUNT];     /* summed kernel durations (timing=1)   */
    uint64_t kernel_launches[SDM_K_COUNT];
    uint64_t items_done;        /* work items finished, this call and earlier
                                   calls of a resumed render                  */
    uint64_t items_total;       /* work items of the render                    */
    uint64_t interface_rays;    /* rays handed across sub-domain interfaces     */
    uint64_t photons_stored;    /* photons of the caustic map                   */
} sdm_stats;

typedef struct {
    float *spectral;            /* [H*W*n_lambda], wavelength fastest, or NULL */
    double *xyz;                /* [H*W*3], or NULL                            */
    int32_t spectral_mem;       /* SDM_MEM_HOST or SDM_MEM_DEVICE              */
    int32_t xyz_mem;
    sdm_stats *stats;           /* host struct, may be NULL                     */
    /* Event signatures (a debug aid for explaining differences against a
     * reference), DEVICE [H*W*n_lambda] or NULL.  Entry (pixel, lambda) is
     * the sum modulo 2^64 of a hash of every event that decides what that
     * pixel's paths contribute at that wavelength: each closest hit (vertex,
     * sample, triangle index or none) and each shadow-ray result (vertex,
     * occluded, or the set of panes crossed), counted where the wavelength's
     * path weight is nonzero.  The hash is the SplitMix64 output function
     * (Steele, Lea and Flood, 2014) of kind << 56 | vertex << 48 | x, with
     * x = sample << 32 | (triangle + 1) for a hit (kind 1), x = 0xFFFF when
     * occluded or else the pane count for a shadow result (kind 2), to which
     * the hashes of 3 << 56 | triangle of every pane crossed are added.  Two
     * renders whose paths decide alike have equal signatures.  Adds two
     * passes per bounce; not with max_items or resume. */
    uint64_t *events;
} sdm_outputs;

/* Context on HIP device `device`.  Owns the work buffers of renders and a
 * second stream of its own (default priority), on which each bounce's
 * shadow walk and accumulation run beside the next bounce's closest-hit
 * pass; a render's results are complete on the caller's stream when the
 * call's work there is.  SDM_SERIAL=1 in the environment when the context is
 * created keeps every pass on the caller's stream (same results).
 * Testing the error paths: with SDM_FAIL_ALLOC=n (n > 0) in the
 * environment when a context is created, the n-th device allocation of the
 * library from then on (any context or scene of the process) fails once,
 * and the call that made it returns SDM_E_NOMEM, with no other effect: the
 * buffer is released, and a later call allocates it again. */
int sdm_context_create(int device, sdm_context **out);
int sdm_context_destroy(sdm_context *ctx);
/* Description of the last failure of a call on ctx (context-owned string). */
const char *sdm_last_error(const sdm_context *ctx);

/* Copies the scene, builds its BVH on the host (binned SAH) and uploads it. */
int sdm_scene_create(sdm_context *ctx, const sdm_scene_desc *desc, sdm_scene **out);
int sdm_scene_destroy(sdm_scene *scene);
/* Geometric sub-domains of a scene: cells along x, y, z (1 1 1 without a
 * cut), the triangle references of all cells (a triangle overlapping several
 * cells counts once per cell) and their BVH nodes.  SDM_E_INVALID for a
 * NULL scene; output pointers may be NULL. */
int sdm_scene_subdomains(const sdm_scene *scene, int32_t cells[3], int64_t *tri_refs, int64_t *nodes);

/* Renders one image: spectral radiance (mean over spp) per pixel and
 * wavelength, and XYZ = sum_i w_i L(lambda_i) cmf(lambda_i) with trapezoid
 * weights w_i in nm.  Geometry and shading run in the requested precision;
 * the per-pixel spectral accumulation and XYZ are FP64.  The call
 * synchronises the stream before it returns: it checks the device flag that
 * reports a full path pool (more glass forks than the pool holds), and in
 * that case renders again with a larger pool (the result is deterministic),
 * returning SDM_E_DEVICE only if the pool cannot grow further. */
int sdm_render(sdm_context *ctx, const sdm_scene *scene, const sdm_render_params *params,
               const sdm_outputs *out, void *hip_stream);

/* Saves the partial render the context holds after SDM_E_ABORTED to a file:
 * a header identifying the render (a digest of the scene's inputs and of the
 * parameters that decide the accumulated values, the resolved tile size and
 * item count), the bitmap of the items done and the FP64 accumulator
 * [H*W*n_lambda] (sums over samples, not yet divided by spp).  SDM_E_INVALID
 * when the context holds no partial render; SDM_E_DEVICE on a file error. */
int sdm_render_checkpoint(sdm_context *ctx, const char *path);

/* Continues a partial render: from the file path written by
 * sdm_render_checkpoint (possibly in another process), or, with path NULL,
 * from the state the context holds after SDM_E_ABORTED.  scene and params
 * must describe the same render (the header's digest is checked:
 * SDM_E_INVALID otherwise); params->max_items applies to the items still to
 * do.  Returns SDM_OK with the whole image in out once every item is done --
 * the same image as one uninterrupted render, up to the order of the FP64
 * additions -- or SDM_E_ABORTED again with the partial image. */
int sdm_render_resume(sdm_context *ctx, const char *path, const sdm_scene *scene,
                      const sdm_render_params *params, const sdm_outputs *out, void *hip_stream);

/* One job of a batch: a scene, its parameters and its outputs. */
typedef struct {
    const sdm_scene *scene;
    const sdm_render_params *params;
    const sdm_outputs *out;
} sdm_job;

/* Renders n_jobs images.  A job of at least half a chunk of paths (W x H x
 * spp x bands; the chunk of jobs[0].params, by default 2^23) fills the
 * device and renders alone; smaller jobs, in their order, are grouped into
 * wavefronts of up to one chunk: the (job x band x tile) work items of a
 * group share one path pool and one kernel sequence per chunk, with a job
 * table giving each path its scene, camera, spectra and accumulator (Sec. 4:
 * dynamic balancing of sub-domains).  Each image equals what sdm_render
 * gives for its job alone.  All jobs must use the same precision, and the
 * jobs of a group that need a network must share one.  A group's chunking,
 * graph replay and pool headroom follow its first job's parameters.  The
 * per-job outputs are as for sdm_render; job statistics are not filled;
 * stats (host, may be NULL) receives the totals.  Synchronises the stream. */
int sdm_render_batch(sdm_context *ctx, int32_t n_jobs, const sdm_job *jobs, sdm_stats *stats,
                     void *hip_stream);

/* Tuning of the wavefront for a scene and parameters: renders twice with
 * each candidate chunk size (2^22, 2^23, 2^24 paths) and pixel tile (8x8,
 * 16x16, 32x32), keeps the fastest, then with those the resident blocks
 * per CU of the closest-hit pass and then of the shadow walk (from the most
 * that fit down to half of it), and uses the choice in later renders of
 * this context with the same scene, image size, wavelength count, depth
 * and precision whose chunk_paths, tile_w, tile_h and blocks per CU are 0.
 * cache_path (may be NULL): a text file of earlier results; a matching entry
 * is taken without measuring, a new result is appended.  The image does not
 * depend on the choice. */
typedef struct {
    int64_t chunk_paths;
    int32_t tile_w, tile_h;
    double ms;                  /* measured time of the chosen render          */
    int32_t from_cache;         /* 1: taken from cache_path                    */
    int32_t trace_blocks_per_cu, shadow_blocks_per_cu;
} sdm_tune_result;

int sdm_autotune(sdm_context *ctx, const sdm_scene *scene, const sdm_render_params *params,
                 const char *cache_path, sdm_tune_result *out, void *hip_stream);

/* Thin-slab optics for m independent inputs (DEVICE arrays of length m):
 * interface Fresnel for n + ik at incidence cos_i, real-Snell path length,
 * Beer-Lambert absorption 4 pi k / lambda + alpha_tint over d_mm, incoherent
 * multiple reflection, s/p averaged.  Writes R and T (DEVICE, length m). */
int sdm_slab_eval(sdm_context *ctx, int64_t m, const float *cos_i, const float *lambda_nm,
                  const float *d_mm, const float *n, const float *k, const float *alpha_tint,
                  float *R, float *T, void *hip_stream);

/* Closest hit of m rays against a scene (DEVICE arrays): o, d [m*3], skip [m]
 * (triangle index to ignore, -1 for none) -> t [m], tri [m] (-1 = miss),
 * uv [m*2] barycentrics.  Hits need t > 1e-6 x scene diagonal; ties in t go
 * to the smaller triangle index. */
int sdm_debug_intersect(sdm_context *ctx, const sdm_scene *scene, int64_t m, const float *o,
                        const float *d, const int32_t *skip, float *t, int32_t *tri, float *uv,
                        void *hip_stream);

/* Sun transmittance from m points (DEVICE arrays o [m*3], skip [m]) at one
 * wavelength: 0 if an opaque triangle lies toward the sun, else the product
 * of the slab transmittances of the panes crossed.  Writes T [m] (DEVICE). */
int sdm_debug_shadow(sdm_context *ctx, const sdm_scene *scene, int64_t m, const float *o,
                     const int32_t *skip, float lambda_nm, float *T, void *hip_stream);

/* Acceleration structures of a scene (for tests and tuning): wide BVH node
 * count, depth (node levels plus leaves) and traversal stack bound; cells and
 * candidate entries of the sun grid (0 and 0 when shadow rays walk the BVH).
 * Any output pointer may be NULL. */
int sdm_scene_info(const sdm_scene *scene, int32_t *n_nodes, int32_t *depth, int32_t *stack,
                   int64_t *grid_cells, int64_t *grid_candidates);

/* ---------------------------------------------------------------------------
 * Bubbly glass (air micro-particles in the glass body, Sec. 1; light
 * scattering as the next material feature, Sec. 6) and its learned surrogate.
 * ------------------------------------------------------------------------- */

/* Monte Carlo of a glass slab holding spherical air bubbles, for m tuples of
 * n_photons photon walks each.  Inputs are DEVICE float arrays of length m:
 * cos_i (incidence cosine, (0, 1]), lambda_nm, d_mm (thickness), rho_b
 * (bubbles per mm^3, >= 0), n, k (optical constants of eq. (1) at lambda),
 * alpha_tint (per mm, may be NULL for 0), n_ref (the real index used inside
 * the slab, may be NULL for n).  Bubble radii are uniform in
 * [rmin_um, rmax_um] micrometres.  A photon meets the entry interface with
 * the complex index (s or p label drawn per photon); inside, directions and
 * decisions use n_ref: Fresnel / total reflection at the faces, Poisson
 * bubbles with extinction rho_b pi <r^2> acting at the collision point with
 * exact sphere optics (outer reflection or p internal reflections, a fresh
 * label per bubble); its weight is exp(-(4 pi k / lambda + alpha_tint) L)
 * over the length L travelled in glass.  Random numbers are Philox4x32-10
 * with counter (tuple0 + i, photon, event, 0x5EB10000 | sub) and key seed.
 * precision: SDM_PREC_FP32 or SDM_PREC_FP64 (the walk's arithmetic; sums are
 * FP64 either way).  Outputs (DEVICE float, length m): R, T (fractions
 * leaving the entry / far face), A (absorbed, may be NULL), w_lobe (RMS angle
 * in radians between the transmitted and the incident direction, weighted
 * by transmitted energy, divided by sqrt(2); 0 when nothing is transmitted).
 * Uses a context-owned FP64 work buffer of 32 m bytes and synchronises the
 * stream before it returns. */
int sdm_slab_mc(sdm_context *ctx, int64_t m, const float *cos_i, const float *lambda_nm,
                const float *d_mm, const float *rho_b, const float *n, const float *k,
                const float *alpha_tint, const float *n_ref, float rmin_um, float rmax_um,
                int32_t n_photons, uint64_t seed, uint32_t tuple0, int32_t precision, float *R,
                float *T, float *A, float *w_lobe, void *hip_stream);

/* sdm_slab_mc for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results as sdm_slab_mc; the FP64 per-tuple
 * sums live in a static device array of the library (2 MiB on each device
 * it runs on, held until the process ends) instead of a context buffer, so
 * m is limited to 65536 tuples (SDM_E_INVALID beyond).  The call allocates
 * nothing and does not synchronise: the outputs are valid once hip_stream
 * is synchronised.  Every call on a device shares that device's array: calls
 * that overlap on one device (other streams, other contexts, other host
 * threads) race and must be serialised by the caller. */
int sdm_slab_mc_noalloc(sdm_context *ctx, int64_t m, const float *cos_i, const float *lambda_nm,
                        const float *d_mm, const float *rho_b, const float *n, const float *k,
                        const float *alpha_tint, const float *n_ref, float rmin_um, float rmax_um,
                        int32_t n_photons, uint64_t seed, uint32_t tuple0, int32_t precision, float *R,
                        float *T, float *A, float *w_lobe, void *hip_stream);

/* Surrogate network of the bubbly slab: 12 -> 64 -> 64 -> 64 -> 3 with ReLU.
 * Input of a tuple (cos_i, lambda_nm, d_mm, rho_b) on pane type p:
 * (cos_i, (lambda - 580) / 200, (d - 3.5) / 1.5, rho_b / 34, E[p][0..7]);
 * outputs o -> R = e^o0 / (e^o0 + e^o1 + 1), T = e^o1 / (same),
 * w = log(1 + e^o2).  Loss: mean over samples of the squared errors of
 * (R, T, w).  Parameters (FP32 master copy, this order):
 *   W1[64][12] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3]
 *   E[n_panes][8]
 * i.e. sdm_mlp_nparams(n_panes) = 9347 + 8 n_panes floats.  Products run on
 * BF16 matrix cores with FP32 accumulation; heads, loss and Adam in FP32. */

typedef struct {
    int32_t steps;      /* Adam steps                                          */
    int32_t batch;      /* samples per step; step s uses rows
                           [(s mod nb) batch, +batch), nb = floor(m / batch)   */
    float lr, beta1, beta2, eps;
} sdm_train_params;

int64_t sdm_mlp_nparams(int32_t n_panes);
/* params: HOST, sdm_mlp_nparams(n_panes) floats; 1 <= n_panes <= 64. */
int sdm_mlp_create(sdm_context *ctx, int32_t n_panes, const float *params, sdm_mlp **out);
int sdm_mlp_destroy(sdm_mlp *mlp);
/* Copies the FP32 master parameters to params (HOST). */
int sdm_mlp_get_params(const sdm_mlp *mlp, float *params);
/* Gradient of the mean loss over m samples with respect to every parameter.
 * tuples [m][4] (cos_i, lambda_nm, d_mm, rho_b), panes [m] (0..n_panes-1),
 * target [m][3] (R, T, w): DEVICE.  grad: DEVICE, nparams floats.  loss:
 * HOST, may be NULL.  Synchronises the stream. */
int sdm_mlp_grad(sdm_mlp *mlp, int64_t m, const float *tuples, const int32_t *panes,
                 const float *target, float *grad, float *loss, void *hip_stream);
/* Adam training on m samples (DEVICE arrays as for sdm_mlp_grad); the
 * optimiser state and its step count persist across calls.  loss_curve:
 * HOST, tp->steps floats (mean batch loss before each step), may be NULL.
 * Synchronises the stream. */
int sdm_mlp_train(sdm_mlp *mlp, int64_t m, const float *tuples, const int32_t *panes,
                  const float *target, const sdm_train_params *tp, float *loss_curve,
                  void *hip_stream);
/* Writes the network to a file: pane count, FP32 master parameters, Adam
 * moments and step count, so that training can continue where it stopped.
 * SDM_E_DEVICE on a file error. */
int sdm_mlp_save(const sdm_mlp *mlp, const char *path);
/* Creates a network in ctx from a file written by sdm_mlp_save (same
 * parameters and optimiser state).  SDM_E_INVALID for a file that is not
 * such a network. */
int sdm_mlp_load(sdm_context *ctx, const char *path, sdm_mlp **out);
/* Pane count (embedding rows) and Adam steps taken; either may be NULL. */
int sdm_mlp_info(const sdm_mlp *mlp, int32_t *n_panes, int64_t *steps);
/* (R, T, w) for m tuples: out [m][3] DEVICE. */
int sdm_mlp_infer(sdm_mlp *mlp, int64_t m, const float *tuples, const int32_t *panes, float *out,
                  void *hip_stream);

/* Error table of the fallback mode: table[pane][c][t][r] (DEVICE float,
 * n_panes * dims[0] * dims[1] * dims[2]) = the largest max(|R - R*|,
 * |T - T*|) between the network and the targets (R*, T*, w*) over the m
 * validation tuples that fall in the cell (0 for empty cells); cells as in
 * sdm_render_params: cos theta in [0, 1], thickness in [2, 5] mm, density in
 * [0, 34] per mm^3, dims[] (HOST) cells each, clamped.  tuples, panes,
 * target: DEVICE as for sdm_mlp_grad.  Synchronises the stream. */
int sdm_mlp_error_table(sdm_mlp *mlp, int64_t m, const float *tuples, const int32_t *panes,
                        const float *target, const int32_t *dims, float *table, void *hip_stream);

/* Matrix-core lane layout check: C32 = A32 B32 with A32 [16][32], B32
 * [32][16] (v_mfma_f32_16x16x32_bf16), C16 = A16 B16 with A16 [16][16],
 * B16 [16][16] (v_mfma_f32_16x16x16_bf16); inputs rounded to BF16; all
 * DEVICE row-major FP32.  Synchronises the stream. */
int sdm_debug_mfma(sdm_context *ctx, const float *A32, const float *B32, float *C32, const float *A16,
                   const float *B16, float *C16, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
