// wavefront.hpp -- host-side launchers of the wavefront kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sdm_types.hpp"

namespace sdm {

template <class R>
void launch_generate(const JobDev *jobs, const BandDev *bands, const ItemDev *items, int n_items, const Work<R> &w,
                     uint64_t total, uint32_t chunk, int grid, hipStream_t s);
template <class R>
void launch_trace(const JobDev *jobs, const Work<R> &w, int cur, int lds_job, bool surface, bool one_job, int grid,
                  hipStream_t s);
template <class R>
void launch_photon_pass(const JobDev *jobs, const PhotonWork<R> &pw, int grid_trace, int num_cu, hipStream_t s);
template <class R>
void launch_caustic(const JobDev *jobs, const BandDev *bands, const Work<R> &w, const PhotonWork<R> &pw, int grid,
                    hipStream_t s);
template <class R>
void launch_dd_trace(const JobDev *jobs, const Work<R> &w, int cur, bool surface, int sweeps, bool march, int grid,
                     hipStream_t s);
template <class R>
void launch_shade(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, bool one_job, int grid,
                  hipStream_t s);
template <class R>
void launch_shade_glass(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, bool one_job, int grid,
                        hipStream_t s);
template <class R>
void launch_bubbly_eval(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, const float *params,
                        const float *E, int n_panes, int grid, hipStream_t s);
template <class R>
void launch_shade_bubbly(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, int grid, hipStream_t s);
template <class R>
void launch_shadow_trace(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int lds_job, bool one_job,
                         int grid, hipStream_t s);
template <class R>
void launch_shadow_accum(const JobDev *jobs, const BandDev *bands, const Work<R> &w, bool one_job, int grid,
                         hipStream_t s);
// Event signatures of the current pool's closest hits and of the shadow
// records (debug; w.sig set).
template <class R>
void launch_sig_hits(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, int grid, hipStream_t s);
template <class R>
void launch_sig_shadow(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int grid, hipStream_t s);
template <class R>
void launch_resample(const float *tab_x, int n_tab, const float *tab_y, int rows, const float *xs, int nl,
                     int stride, R *out, hipStream_t s);
// Resident blocks of 256 threads per CU of a render kernel (SDM_K_* class)
// with lds_bytes of dynamic LDS.
template <class R>
int occupancy(int kernel_class, int lds_bytes = 0);

void launch_finalize(const double *acc, int64_t npix, int nl, int spp, const double *wts, const double *cmf,
                     float *spec, double *xyz, hipStream_t s);
void launch_zero_f64(double *a, int64_t n, hipStream_t s);
void launch_zero_counters(Counters *c, hipStream_t s);
void launch_advance_cursor(Counters *c, uint32_t chunk, hipStream_t s);
void launch_reset_records(Counters *c, hipStream_t s);
void launch_slab_eval(int64_t m, const float *c, const float *lam, const float *d, const float *n, const float *k,
                      const float *tint, float *R, float *T, hipStream_t s);
void launch_debug_intersect(const SceneDev &sc, uint32_t m, const float *o, const float *d, const int32_t *skip,
                            const int32_t *orig_to_leaf, float *t, int32_t *tri, float *uv,
                            int32_t *gstack, int grid, hipStream_t s);
void launch_debug_shadow(const SceneDev &sc, uint32_t m, const float *o, const int32_t *skip,
                         const int32_t *orig_to_leaf, float lambda_nm, const float *n_at, const float *k_at,
                         const float *t_at, float *T, int32_t *gstack, int grid, hipStream_t s);
int block_size();
// Threads per block of the closest-hit traversal kernel.
int trace_block_size();

}  // namespace sdm
