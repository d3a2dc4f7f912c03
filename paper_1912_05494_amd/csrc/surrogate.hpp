// surrogate.hpp -- launchers of the bubbly-slab Monte Carlo and of the
// surrogate network kernels (surrogate.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdm {

constexpr int kMaxPanes = 64;   // embedding rows (glass types) a network can hold

void launch_mfma_probe(const float *A32, const float *B32, float *C32, const float *A16, const float *B16, float *C16,
                       hipStream_t s);

// Static device scratch of the allocation-free slab Monte Carlo: its
// tuple capacity, the devices it is resolved for, and the device address on
// `device` (which must be current); returns 0, or -1 on failure.
constexpr uint32_t kMcScratchTuples = 1u << 16;
constexpr int kMcScratchDevices = 64;
int mc_scratch_address(int device, double **out);

template <class R>
void launch_slab_mc(uint32_t m, uint32_t nph, const float *cos_i, const float *lam, const float *d, const float *rho,
                    const float *n, const float *k, const float *tint, const float *n_ref, double r2_mm,
                    uint64_t seed, uint32_t tuple0, double *acc, float *Rr, float *Tt, float *A, float *W, int num_cu,
                    hipStream_t s);

void launch_mlp_pack(const float *params, void *wb, float *bb, hipStream_t s);
void launch_mlp_grad(uint32_t m, int n_panes, const float *tup, const int32_t *pane, const float *target,
                     const void *wb, const float *bb, const float *E, float inv_n, float *partial, float *loss_partial,
                     int *bad, int nblk, hipStream_t s);
void launch_mlp_reduce(int nblk, int P, const float *partial, const float *loss_partial, float inv_n, float *grad,
                       float *loss, hipStream_t s);
// Sum of the gradient pass's block rows, Adam step and the new parameters'
// kernel copies (wb, bb) in one launch; loss receives the mean loss.
void launch_mlp_reduce_adam(int nblk, int P, const float *partial, const float *loss_partial, float inv_n, float *loss,
                            float *params, float *m1, float *m2, float lr, float b1, float b2, float eps, float c1,
                            float c2, void *wb, float *bb, hipStream_t s);
void launch_mlp_infer(uint32_t m, int n_panes, const float *tup, const int32_t *pane, const void *wb, const float *bb,
                      const float *E, float *out, int *bad, int num_cu, hipStream_t s);
void launch_zero_i32(int *p, int n, hipStream_t s);
void launch_err_cells(uint32_t m, const float *tup, const int32_t *pane, const float *y, const float *target,
                      int n_panes, const int dims[3], float *table, int *bad, hipStream_t s);
int mlp_net_params();
int mlp_wb_elems();
int mlp_bb_elems();

}  // namespace sdm
