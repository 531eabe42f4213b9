// Per-row device helpers shared by the 2D and 3D sweeps and the adjoints:
// float4 rows, the projection onto the lam-disc, lane exchanges by DPP,
// float64 wave and block reductions, and agent-scope loads and stores of
// the reduction partials.
#pragma once

#include "common.h"
#include "pointwise.h"

namespace tvpd {
namespace dev {

struct F4 {
  float v[4];
};

__device__ __forceinline__ F4 ld4(const float* p) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  F4 r;
  r.v[0] = t.x;
  r.v[1] = t.y;
  r.v[2] = t.z;
  r.v[3] = t.w;
  return r;
}

__device__ __forceinline__ void st4(float* p, const F4& a) {
  *reinterpret_cast<float4*>(p) = make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
}

__device__ __forceinline__ F4 zero4() {
  F4 r;
#pragma unroll
  for (int j = 0; j < 4; ++j) r.v[j] = 0.0f;
  return r;
}

// Projection of q onto the disc of radius lam.
__device__ __forceinline__ void project2(float qx, float qy, float lam,
                                         float& px, float& py) {
  const float c = ball_scale(sq2(qx, qy), lam);
  px = qx * c;
  py = qy * c;
}

// Value of the next (from_right) or previous (from_left) lane of the wave,
// by a DPP wavefront shift (wave_shl:1 / wave_shr:1): a VALU operation with
// no LDS round trip, unlike a bpermute shuffle.  The edge lane keeps its own
// value, as a shuffle past the wave's end does; callers replace it.  All
// lanes of the wave must be active.
__device__ __forceinline__ float from_right(float v) {
  const int x = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_left(float v) {
  const int x = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x138, 0xF, 0xF, false));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum (a, b) over the block in a fixed order; result valid in thread 0.
// red: two rows of NW >= blockDim.x / 64 slots in LDS.
template <int NW>
__device__ __forceinline__ void block_sum2(double& a, double& b, double (*red)[NW]) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < nw; ++w) {
      sa += red[0][w];
      sb += red[1][w];
    }
    a = sa;
    b = sb;
  }
}

__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace dev
}  // namespace tvpd
