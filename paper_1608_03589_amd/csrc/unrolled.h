// Unrolled (differentiable) solver: planes, plan and kernel launchers.
#pragma once

#include "common.h"

namespace tvpd {

// Plane block of one image of an unrolled workspace; image b's plane `id`
// starts at base + b * istride + id * plane.
struct PlaneSet {
  float* base;
  int64_t istride;  // floats per image block
  int64_t plane;    // floats per plane
  int32_t nb;       // images
  int32_t ndim;
  int32_t nz, ny, nx, pitch;
};

// One forward step k -> k+1 (per-iteration coefficients from device memory).
struct StepIds {
  int fk, fkm, pk;  // inputs (pk: first of ndim planes)
  int fn, pn;       // outputs
};

// A forward pass k -> k+n in 2D (n <= kMaxPass): the outputs of every
// iteration k+s at index s-1.
struct PassIds {
  int fk, fkm, pk;
  int fn[kMaxPass], pn[kMaxPass];
};

// One adjoint step.
struct AdjIds {
  int fk, fkm, pk;      // forward state of step k
  int g;
  int a_in, b_in, r_in;   // adjoint inputs (r: ndim planes)
  int a_out, b_out, t_out;  // adjoint outputs (t: ndim planes, next r)
  int pn;               // scratch: recomputed p^{k+1} (ndim planes)
  int gbar;             // accumulated dL/dg
};

hipError_t launch_u_init(const PlaneSet& P, const float* g, int id_g,
                         int id_zero, int nzero, hipStream_t s);
// 3D only: one iteration k -> k+1.
hipError_t launch_u_step(const PlaneSet& P, const StepIds& ids,
                         const float* coeffs, int k, float theta,
                         hipStream_t s);
// 2D only: iterations k .. k+n-1 in one launch (1 <= n <= kMaxPass).
hipError_t launch_u_pass2d(const PlaneSet& P, const PassIds& ids,
                           const float* coeffs, int k, int n, float theta,
                           hipStream_t s);
hipError_t launch_u_read(const PlaneSet& P, int id, float* out, hipStream_t s);
hipError_t launch_u_load(const PlaneSet& P, const float* in, int id,
                         hipStream_t s);
hipError_t launch_u_zero(const PlaneSet& P, int id, int n, hipStream_t s);
hipError_t launch_u_adjoint(const PlaneSet& P, const AdjIds& ids,
                            const float* coeffs, int k, float theta,
                            double* partials, int64_t max_partials,
                            float* grad_coeffs, hipStream_t s);
hipError_t launch_u_final_grad(const PlaneSet& P, int gbar, int a, int b,
                               float* grad_g, hipStream_t s);
int64_t u_partials_needed(const PlaneSet& P);
bool fused_adjoint_enabled();  // unrolled_api.hip

}  // namespace tvpd
