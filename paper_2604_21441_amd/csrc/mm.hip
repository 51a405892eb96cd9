// MM point charges as an extra per-atom network input (electrostatic
// embedding through the model, with forces on MM atoms; Methods: the 2026
// interface passes MM positions and charges, and the model may put forces on
// MM atoms):
//   phi_i = ke * sum_j q_j fc(r_ij; Rm) / r_ij     over MM atoms j, r_ij < Rm
// The pass is all-pairs over (NNP atom, MM atom): one lane per MM atom; the
// grid's second dimension splits the NNP atoms into chunks of kNnpChunk, so
// that a small ML region still gives many wavefronts, and each wavefront
// walks its chunk (unrolled, so that the reductions of several atoms are in
// flight together) and reduces each atom's sum across lanes.  Intended for ML
// regions of up to a few thousand atoms.
#include "nnp_internal.h"

namespace nnp {
namespace {

constexpr int kBlock = 256;
constexpr int kNnpChunk = 16;   // NNP atoms per wavefront

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void mm_disp(const float4& pi, float yx, float yy, float yz, const Geometry& g,
                                        float& dx, float& dy, float& dz, float& r2) {
  dx = yx - pi.x; dy = yy - pi.y; dz = yz - pi.z;
  if (g.periodic) {
    dx -= g.box[0] * rintf(dx * g.inv_box[0]);
    dy -= g.box[1] * rintf(dy * g.inv_box[1]);
    dz -= g.box[2] * rintf(dz * g.inv_box[2]);
  }
  r2 = dx * dx + dy * dy + dz * dz;
}

__global__ __launch_bounds__(kBlock) void k_fill_f64(double* p, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_mm_fwd(const float4* __restrict__ spos, int n,
                                                   const float* __restrict__ mm_pos,
                                                   const float* __restrict__ mm_q, int n_mm,
                                                   DescParams p, Geometry g, double* __restrict__ phi) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int lane = threadIdx.x & 63;
  bool ok = j < n_mm;
  float yx = 0.f, yy = 0.f, yz = 0.f, q = 0.f;
  if (ok) {
    yx = mm_pos[3 * (int64_t)j]; yy = mm_pos[3 * (int64_t)j + 1]; yz = mm_pos[3 * (int64_t)j + 2];
    q = mm_q[j];
  }
  const float rm2 = p.mm_cutoff * p.mm_cutoff;
  const float inv2rm = 0.5f / p.mm_cutoff;
  const int i0 = blockIdx.y * kNnpChunk, i1 = min(n, i0 + kNnpChunk);
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    float4 pi = spos[i];
    float dx, dy, dz, r2;
    mm_disp(pi, yx, yy, yz, g, dx, dy, dz, r2);
    float t = 0.f;
    if (ok && r2 < rm2) {
      float ir = __builtin_amdgcn_rsqf(r2);
      float r = r2 * ir;
      float fc = 0.5f * __builtin_amdgcn_cosf(r * inv2rm) + 0.5f;
      t = q * fc * ir;
    }
    t = wave_sum(t);
    if (lane == 0 && t != 0.f) unsafeAtomicAdd(&phi[i], (double)t);
  }
}

__global__ __launch_bounds__(kBlock) void k_mm_finish(const double* __restrict__ phi, int n, DescParams p,
                                                      float* __restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[(int64_t)i * p.stride + p.D] = (float)(p.ke * phi[i]);
}

// Adjoint: dE/dphi_i = g[i][D] (+ the predicted charge q_i of a network with
// a charge output, whose energy holds q_i phi_i);  dphi_i/dy_j = ke q_j f'(r) u,  f(r) = fc(r)/r,
// u = (y_j - x_i)/r.  MM atom j gets -sum_i dE/dphi_i dphi_i/dy_j (owned by its
// lane), NNP atom i gets the opposite of its column sum (wave-reduced, one
// FP64 atomic per wavefront and atom).
__global__ __launch_bounds__(kBlock) void k_mm_bwd(const float4* __restrict__ spos,
                                                   const int* __restrict__ slot_atom, int n,
                                                   const float* __restrict__ mm_pos,
                                                   const float* __restrict__ mm_q, int n_mm,
                                                   const float* __restrict__ gx,
                                                   const float* __restrict__ qpred, DescParams p, Geometry g,
                                                   double* __restrict__ forces,
                                                   double* __restrict__ mm_forces,
                                                   double* __restrict__ link_forces) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int lane = threadIdx.x & 63;
  bool ok = j < n_mm;
  float yx = 0.f, yy = 0.f, yz = 0.f, q = 0.f;
  if (ok) {
    yx = mm_pos[3 * (int64_t)j]; yy = mm_pos[3 * (int64_t)j + 1]; yz = mm_pos[3 * (int64_t)j + 2];
    q = mm_q[j];
  }
  const float rm2 = p.mm_cutoff * p.mm_cutoff;
  const float inv2rm = 0.5f / p.mm_cutoff;
  const float dfc_s = -0.5f * 3.14159265358979323846f / p.mm_cutoff;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  const int i0 = blockIdx.y * kNnpChunk, i1 = min(n, i0 + kNnpChunk);
#pragma unroll 4
  for (int i = i0; i < i1; ++i) {
    float4 pi = spos[i];
    float gi = gx[(int64_t)i * p.stride + p.D];
    if (qpred != nullptr) gi += qpred[i];
    float dx, dy, dz, r2;
    mm_disp(pi, yx, yy, yz, g, dx, dy, dz, r2);
    float vx = 0.f, vy = 0.f, vz = 0.f;
    if (ok && r2 < rm2) {
      float ir = __builtin_amdgcn_rsqf(r2);
      float r = r2 * ir;
      float arg = r * inv2rm;
      float fc = 0.5f * __builtin_amdgcn_cosf(arg) + 0.5f;
      float dfc = dfc_s * __builtin_amdgcn_sinf(arg);
      float fp = (dfc - fc * ir) * ir;            // d/dr (fc / r)
      float w = (float)p.ke * gi * q * fp * ir;   // times u = d / r
      vx = w * dx; vy = w * dy; vz = w * dz;
    }
    fx -= vx; fy -= vy; fz -= vz;
    float sx = wave_sum(vx), sy = wave_sum(vy), sz = wave_sum(vz);
    if (lane == 0 && (sx != 0.f || sy != 0.f || sz != 0.f)) {
      const int a = slot_atom[i];   // a < 0: link atom -1 - a
      double* f = a >= 0 ? forces + 3 * (int64_t)a : link_forces + 3 * (int64_t)(-1 - a);
      unsafeAtomicAdd(f + 0, (double)sx);
      unsafeAtomicAdd(f + 1, (double)sy);
      unsafeAtomicAdd(f + 2, (double)sz);
    }
  }
  if (ok && mm_forces != nullptr) {   // one NNP chunk: this lane owns the row; else several chunks add
    double* f = mm_forces + 3 * (int64_t)j;
    if (gridDim.y == 1) {
      f[0] += fx; f[1] += fy; f[2] += fz;
    } else if (fx != 0.0 || fy != 0.0 || fz != 0.0) {
      unsafeAtomicAdd(f + 0, fx);
      unsafeAtomicAdd(f + 1, fy);
      unsafeAtomicAdd(f + 2, fz);
    }
  }
}

}  // namespace

hipError_t launch_mm_fwd(nnp_model& m, int n, int n_mm, const float* mm_pos, const float* mm_q,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, m.d_phi, n);
  if (n_mm > 0) {
    hipLaunchKernelGGL(k_mm_fwd, dim3((n_mm + kBlock - 1) / kBlock, (n + kNnpChunk - 1) / kNnpChunk), dim3(kBlock),
                       0, st, m.d_spos, n, mm_pos, mm_q, n_mm, m.dp, m.geo, m.d_phi);
  }
  hipLaunchKernelGGL(k_mm_finish, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, m.d_phi, n, m.dp,
                     m.d_x);
  return hipGetLastError();
}

hipError_t launch_mm_bwd(nnp_model& m, int n, int n_mm, const float* mm_pos, const float* mm_q,
                         double* forces, double* mm_forces, hipStream_t st) {
  if (n == 0 || n_mm == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mm_bwd, dim3((n_mm + kBlock - 1) / kBlock, (n + kNnpChunk - 1) / kNnpChunk), dim3(kBlock),
                     0, st, m.d_spos, m.d_slot_atom, n, mm_pos, mm_q, n_mm, m.d_g, m.charges ? m.d_q : nullptr, m.dp,
                     m.geo, forces, mm_forces, m.d_link_F);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p, (int)n);
  return hipGetLastError();
}

}  // namespace nnp
