// Mechanical embedding (Theory, eq. 3): the ML-MM coupling left at the MM
// level, Coulomb plus 12-6 Lennard-Jones between every ML atom and every MM
// atom with fixed force-field charges and LJ parameters:
//   E = sum_{i in ML} sum_{j in MM, r < rc} ke q_i q_j / r + 4 eps_ij ((s_ij/r)^12 - (s_ij/r)^6)
// with Lorentz-Berthelot mixing s_ij = (s_i + s_j)/2, eps_ij = sqrt(eps_i eps_j).
//
// One lane per MM atom; the ML atoms (a small region) are staged in LDS in
// chunks and every lane walks them.  Each pair is evaluated in FP32; the MM
// atom's force and the lane's energy accumulate in FP64 registers; an ML
// atom's force is reduced over the wavefront and added with one FP64 atomic
// per wavefront (skipped when no lane of the wavefront is inside the cutoff).
#include "nnp_internal.h"

namespace nnp {
namespace {

constexpr int kMeBlock = 256;
constexpr int kMeChunk = 256;   // ML atoms per LDS chunk

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wsum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(kMeBlock) void k_me_pairs(const float* __restrict__ ml_pos,
                                                       const float* __restrict__ ml_par, int n_ml,
                                                       const float* __restrict__ mm_pos,
                                                       const float* __restrict__ mm_par, int n_mm, Geometry g,
                                                       float rc2, float ke, double* __restrict__ energy,
                                                       double* __restrict__ ml_f, double* __restrict__ mm_f,
                                                       int accumulate) {
  __shared__ float4 sx[kMeChunk];   // ML x, y, z, q
  __shared__ float2 sp[kMeChunk];   // ML sigma, eps
  const int j = blockIdx.x * kMeBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool ok = j < n_mm;
  float yx = 0.f, yy = 0.f, yz = 0.f, qj = 0.f, sj = 0.f, ej = 0.f;
  if (ok) {
    yx = mm_pos[3 * (int64_t)j];
    yy = mm_pos[3 * (int64_t)j + 1];
    yz = mm_pos[3 * (int64_t)j + 2];
    qj = mm_par[3 * (int64_t)j];
    sj = mm_par[3 * (int64_t)j + 1];
    ej = mm_par[3 * (int64_t)j + 2];
  }
  double fx = 0.0, fy = 0.0, fz = 0.0, eacc = 0.0;
  for (int c0 = 0; c0 < n_ml; c0 += kMeChunk) {
    const int nc = min(kMeChunk, n_ml - c0);
    __syncthreads();
    for (int t = threadIdx.x; t < nc; t += kMeBlock) {
      const int i = c0 + t;
      sx[t] = make_float4(ml_pos[3 * (int64_t)i], ml_pos[3 * (int64_t)i + 1], ml_pos[3 * (int64_t)i + 2],
                          ml_par[3 * (int64_t)i]);
      sp[t] = make_float2(ml_par[3 * (int64_t)i + 1], ml_par[3 * (int64_t)i + 2]);
    }
    __syncthreads();
    for (int t = 0; t < nc; ++t) {
      const float4 xi = sx[t];
      float dx = yx - xi.x, dy = yy - xi.y, dz = yz - xi.z;
      if (g.periodic) {
        dx -= g.box[0] * rintf(dx * g.inv_box[0]);
        dy -= g.box[1] * rintf(dy * g.inv_box[1]);
        dz -= g.box[2] * rintf(dz * g.inv_box[2]);
      }
      const float r2 = dx * dx + dy * dy + dz * dz;
      const bool in = ok && r2 < rc2;
      float vx = 0.f, vy = 0.f, vz = 0.f;
      if (in) {
        const float2 pi = sp[t];
        const float ir2 = 1.f / r2;
        const float ir = sqrtf(ir2);
        const float qq = ke * xi.w * qj;
        const float s = 0.5f * (pi.x + sj);
        const float eps = sqrtf(pi.y * ej);
        const float s2 = s * s * ir2;
        const float s6 = s2 * s2 * s2;
        const float s12 = s6 * s6;
        const float ec = qq * ir;
        eacc += (double)ec + (double)(4.f * eps * (s12 - s6));
        const float w = (ec + eps * (48.f * s12 - 24.f * s6)) * ir2;   // -dE/dr / r
        vx = w * dx;
        vy = w * dy;
        vz = w * dz;
        fx += vx;
        fy += vy;
        fz += vz;
      }
      if (__ballot(in) != 0) {
        const float rx = wsum(vx), ry = wsum(vy), rz = wsum(vz);
        if (lane == 0) {
          double* f = ml_f + 3 * (int64_t)(c0 + t);
          unsafeAtomicAdd(f + 0, -(double)rx);
          unsafeAtomicAdd(f + 1, -(double)ry);
          unsafeAtomicAdd(f + 2, -(double)rz);
        }
      }
    }
  }
  if (ok) {
    double* f = mm_f + 3 * (int64_t)j;
    if (accumulate) {
      fx += f[0];
      fy += f[1];
      fz += f[2];
    }
    f[0] = fx;
    f[1] = fy;
    f[2] = fz;
  }
  eacc = wsum_d(eacc);
  if (lane == 0 && eacc != 0.0) unsafeAtomicAdd(energy, eacc);
}

}  // namespace

hipError_t launch_me_pairs(int n_ml, const float* ml_pos, const float* ml_par, int n_mm, const float* mm_pos,
                           const float* mm_par, const Geometry& g, float cutoff, float ke, double* energy,
                           double* ml_f, double* mm_f, int accumulate, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (!accumulate) {
    e = launch_fill_f64(energy, 1, st);
    if (e == hipSuccess) e = launch_fill_f64(ml_f, 3 * (int64_t)n_ml, st);
    if (e != hipSuccess) return e;
  }
  if (n_mm == 0) return hipSuccess;
  const float rc2 = cutoff > 0.f ? cutoff * cutoff : INFINITY;
  hipLaunchKernelGGL(k_me_pairs, dim3((n_mm + kMeBlock - 1) / kMeBlock), dim3(kMeBlock), 0, st, ml_pos, ml_par,
                     n_ml, mm_pos, mm_par, n_mm, g, rc2, ke, energy, ml_f, mm_f, accumulate);
  return hipGetLastError();
}

}  // namespace nnp
