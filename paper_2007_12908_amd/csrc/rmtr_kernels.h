// Host-side launch interface of the HIP kernels (internal to librmtr).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "rmtr_device.h"

namespace rmtr {

// Scratch for deterministic two-stage reductions: partial sums of at most
// kMaxPartials blocks, then one block sums them in a fixed order.
constexpr int kMaxPartials = 4096;

struct ElemArgs {
  int dim;
  int N;           // cells per side on this level
  double h;
  MatP<double> m;
  const uint8_t* dir;  // per-node Dirichlet bits, or null (default set)
  // ring partials and seam slots of the FP64 3D gradient and Hv on
  // non-overlapping tiles (ring_values(N) doubles at least), or null:
  // overlapping tiles
  double* ring = nullptr;
};

// doubles of the ring partials and seam slots that the gradient and Hv of
// a 3D level of N cells per side (or of any coarser level) need
size_t ring_values(int N);

// ---- element kernels (elem_kernels.hip)
// workgroups of the energy kernel = partial sums it writes (<= kMaxPartials)
int energy_partials(const ElemArgs& a);
hipError_t launch_energy(const ElemArgs& a, const double* x, const void* s, int s_fp32, const double* p,
                         double* partials, double* out, hipStream_t st);
hipError_t launch_gradient(const ElemArgs& a, const double* x, const double* p, double* g, hipStream_t st);
hipError_t launch_hessvec(const ElemArgs& a, const void* xl, const void* p, const void* v, void* hv,
                          int fp32, hipStream_t st);
hipError_t launch_diag_blocks(const ElemArgs& a, const void* xl, const void* p, void* D, int fp32,
                              hipStream_t st);
hipError_t launch_reduce_partials(const double* partials, int n, double* out, hipStream_t st);

// ---- assembled block stencils (stencil_kernels.hip)
size_t stencil_values(int dim, int N);
size_t coef_values(int dim, int N, int split);  // split: MatP::split
// lagged Hessian at xl (FP64 arithmetic) -> stencil S (double, or float if fp32);
// coef: scratch of coef_values doubles
hipError_t launch_st_assemble(const ElemArgs& a, const double* xl, const double* p, double* coef, void* S,
                              int fp32, hipStream_t st);
hipError_t launch_em_to_st(int dim, int N, const double* K, void* S, int fp32, hipStream_t st);
// Galerkin coarse stencil Sc (level with Nf/2 cells, FP64) = R Sf I of the
// fine stencil Sf (FP64, or FP32 if fp32), rows and columns of the coarse
// Dirichlet dofs (mask dirc, null: default set) zero; work holds
// st_rap_work_doubles(dim, Nf, fp32) doubles (the intermediate stencils are
// kept in the fine stencil's precision)
size_t st_rap_work_doubles(int dim, int Nf, int fp32);
hipError_t launch_st_rap(int dim, int Nf, const void* Sf, int fp32, double* Sc, const uint8_t* dirc, double* work,
                         hipStream_t st);
hipError_t launch_st_matvec(int dim, int N, const void* S, const void* v, void* y, int fp32, hipStream_t st);
hipError_t launch_st_pgs(int dim, int N, const void* S, const uint8_t* dir, const void* g, const void* lo,
                         const void* hi, void* s, int n_sweeps, int fp32, hipStream_t st);
// Gershgorin row sums of |S| (as -min in slot 4) and g^T g (slot 0): five
// partial values per block, block count returned in nblocks_out (<= 1024)
hipError_t launch_st_rowabs(int dim, int N, const double* S, const double* gv, double* partials, int* nblocks_out,
                            hipStream_t st);

// ---- transfers (transfer_kernels.hip)
hipError_t launch_prolong(int dim, int Nc, const void* xc, void* xf, int fp32, hipStream_t st);
hipError_t launch_restrict(int dim, int Nc, int mode, const void* xf, void* xc, int fp32, hipStream_t st);

// ---- fields (fields_kernels.hip)
hipError_t launch_init_fields(int dim, int N, const double* table, int n_frac, double band, int p_mode,
                              double p_value, double p_band, double* c0, double* p, hipStream_t st);

// ---- Neumann boundary load (boundary_kernels.hip)
// traction per face (face = 2 axis + side), constant on the face
struct NeumannTraction {
  double t[6][3];
};
// b = int_{Gamma_N} (tbar + p n) N ds on the u components of the faces in
// face_mask (bit f = face f), 0 elsewhere (c components included)
hipError_t launch_neumann_load(int dim, int N, int face_mask, const NeumannTraction& tr, const double* p, double* b,
                               hipStream_t st);

// ---- vector kernels (linalg_kernels.hip)
hipError_t launch_dot(int64_t n, const double* a, const double* b, double* partials, double* out,
                      hipStream_t st);
// out = max_i |a_i| (device scalar)
hipError_t launch_amax(int64_t n, const double* a, double* partials, double* out, hipStream_t st);
hipError_t launch_chi(int dim, int N, const double* x, const double* g, const double* c_lower,
                      const uint8_t* dir, double* partials, double* out, hipStream_t st);
hipError_t launch_axpy(int64_t n, double alpha, const double* x, double* y, hipStream_t st);
hipError_t launch_step_box(int dim, int N, const double* x, const double* Lb, const double* Ub, double delta,
                           const uint8_t* dir, double* lo, double* hi, hipStream_t st);
hipError_t launch_fine_bounds(int dim, int N, const double* c_lower, double* Lb, double* Ub,
                              hipStream_t st);
hipError_t launch_convert(int64_t n, const void* src, int src_fp32, void* dst, int dst_fp32, hipStream_t st);
hipError_t launch_add_scaled(int64_t n, const double* a, double alpha, const double* b, double beta,
                             const double* c, double* out, hipStream_t st);
hipError_t launch_zero_masked(int dim, int N, double* v, const uint8_t* dir, hipStream_t st);
hipError_t launch_fill(int64_t n, double v, double* out, hipStream_t st);
hipError_t launch_clamp(int64_t n, const double* lo, const double* hi, double* s, hipStream_t st);
hipError_t launch_inject_scalar(int dim, int Nc, const double* fine, double* coarse, hipStream_t st);
// per-node Dirichlet bits of a coarse level: those of the fine node it
// coincides with (fine node (2i, 2j, 2k) -> coarse node (i, j, k))
hipError_t launch_inject_mask(int dim, int Nc, const uint8_t* fine, uint8_t* coarse, hipStream_t st);
hipError_t launch_any_nonzero(int64_t n, const double* v, int* flag, hipStream_t st);

// ---- MPRGP (mprgp.hip)
struct MprgpResult {
  int iterations;
  int status;  // 0 converged, 1 max iterations, 2 negative curvature (fallback applied)
};
// S: the level's assembled block stencil (FP64); host_scalars: at least 10
// doubles of host-mapped coherent memory (slots 0-4 take reduced scalars,
// slot 8 a pass sequence word)
hipError_t run_mprgp(int dim, int N, const double* S, const uint8_t* dir, const double* g, const double* lo,
                     const double* hi, double* s, int max_it, double rtol, int fallback_sweeps, double* work,
                     double* host_scalars, MprgpResult* res, hipStream_t st);
size_t mprgp_work_doubles(int dim, int N);

// ---- learned proposal network (cnn_kernels.hip)
// channels 8 -> 32 -> 32 -> 32 -> 32 -> 32 -> 4; weights BF16 [27][Cin][Cout]
// per layer, concatenated; biases FP32, concatenated; tensors channels-last
int64_t nn_weight_count();
int64_t nn_bias_count();
int64_t nn_act_floats(int64_t nvox);  // all seven layer tensors of one box
void nn_layers(float* act, int64_t nvox, float* layer[7]);
hipError_t nn_forward(const uint16_t* w, const float* bias, float* const layer[7], int nx, int ny, int nz,
                      hipStream_t st);
size_t nn_backward_work_floats(int64_t nvox);
hipError_t nn_backward(const uint16_t* w, const float* act, const float* dout, float* dw, float* db, int nx, int ny,
                       int nz, float* work, hipStream_t st);
hipError_t nn_mse(const float* out, const float* target, float* dout, int nx, int ny, int nz, const int* window,
                  double* partials, double* loss_dev, hipStream_t st);
hipError_t nn_adam(int64_t n, int64_t n_bf16, float lr, int t, const float* g, float* p, float* m, float* v,
                   uint16_t* pbf, hipStream_t st);
hipError_t nn_to_bf16(int64_t n, const float* a, uint16_t* b, hipStream_t st);
// per-component RMS of the nodal 4-vector g (partials: kMaxPartials doubles)
hipError_t nn_grad_rms(int64_t nn, const double* g, double* partials, double* rms, hipStream_t st);
hipError_t nn_features(int64_t nn, const double* x, const double* g, const float* scales, const double* rms,
                       float* feat, hipStream_t st);
hipError_t nn_proposal(int64_t n, const float* out, const float* scales, const double* rms, const double* lo,
                       const double* hi, double* s, hipStream_t st);
// training target s_k / (scales[8+k] rms_k) of a step s (n values, 4 per node)
hipError_t nn_target(int64_t n, const double* s, const float* scales, const double* rms, float* t, hipStream_t st);
// the 12 normalisation constants from ns samples' RMS values (12 per sample)
hipError_t nn_fit_scales(int ns, const double* rms_samples, float* scales, hipStream_t st);

}  // namespace rmtr
