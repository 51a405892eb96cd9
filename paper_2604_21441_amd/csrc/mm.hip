// MM point charges as an extra per-atom network input (electrostatic
// embedding through the model, with forces on MM atoms; Methods: the 2026
// interface passes MM positions and charges, and the model may put forces on
// MM atoms):
//   phi_i = ke * sum_j q_j fc(r_ij; Rm) / r_ij     over MM atoms j, r_ij < Rm
// The pass is all-pairs over (NNP atom, MM atom).  A workgroup takes a row of
// kNnpChunk NNP atoms (grid y) and a range of MM atoms, one per lane (grid x,
// at most kMaxMmBlocks workgroups; more MM atoms loop); each lane keeps one
// running sum per NNP atom of the row, and after its MM atoms the sums are
// reduced across lanes (a DPP transposing butterfly within each 16-lane row:
// 15 exchanges for all 16 sums, where a shuffle tree per sum took 96 LDS
// round trips) and wavefronts, and stored as the workgroup's partial.
// A second launch adds the partials of every NNP atom in a fixed order (FP64).
// No atomics on the NNP side: with a small ML region every NNP atom collects
// a term from each of hundreds of workgroups, and FP64 atomics on one address
// serialise (60 NNP atoms, 30,000 charges: 10.9 us forward and 15.7 us
// adjoint with per-wavefront atomics).  Intended for ML regions of up to a
// few thousand atoms.
#include "nnp_internal.h"

namespace nnp {
namespace {

constexpr int kBlock = 256;
constexpr int kNnpChunk = 16;       // NNP atoms per workgroup row (= lanes of a DPP row)
constexpr int kMaxMmBlocks = 512;   // workgroups along the MM atoms

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// v[0 .. 16) summed over the 16 lanes of each DPP row: lane l of a row ends
// with the row's total of value l & 15 in v[0].
__device__ __forceinline__ void row_sum16(float* v, int lane) {
  halve<8, kDppMirror>(v, lane & 8);
  halve<4, kDppHalfMirror>(v, lane & 4);
  halve<2, kDppXor2>(v, lane & 2);
  halve<1, kDppXor1>(v, lane & 1);
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

// part[i * gridDim.x + blockIdx.x] = this workgroup's share of phi_i / ke.
__global__ __launch_bounds__(kBlock) void k_mm_fwd(const float4* __restrict__ spos, int n,
                                                   const float* __restrict__ mm_pos,
                                                   const float* __restrict__ mm_q, int n_mm,
                                                   DescParams p, Geometry g, float* __restrict__ part) {
  __shared__ float red[kBlock / kNnpChunk][kNnpChunk];   // [wavefront row][NNP atom]
  const int lane = threadIdx.x & 63;
  const int i0 = blockIdx.y * kNnpChunk, cnt = min(n - i0, kNnpChunk);
  const float rm2 = p.mm_cutoff * p.mm_cutoff;
  const float inv2rm = 0.5f / p.mm_cutoff;
  float acc[kNnpChunk];
#pragma unroll
  for (int c = 0; c < kNnpChunk; ++c) acc[c] = 0.f;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < n_mm; j += gridDim.x * kBlock) {
    const float yx = mm_pos[3 * (int64_t)j], yy = mm_pos[3 * (int64_t)j + 1], yz = mm_pos[3 * (int64_t)j + 2];
    const float q = mm_q[j];
#pragma unroll
    for (int c = 0; c < kNnpChunk; ++c) {
      if (c < cnt) {
        const float4 pi = spos[i0 + c];
        float dx, dy, dz, r2;
        mm_disp(pi, yx, yy, yz, g, dx, dy, dz, r2);
        if (r2 < rm2) {
          float ir = __builtin_amdgcn_rsqf(r2);
          float r = r2 * ir;
          float fc = 0.5f * __builtin_amdgcn_cosf(r * inv2rm) + 0.5f;
          acc[c] += q * fc * ir;
        }
      }
    }
  }
  row_sum16(acc, lane);
  red[threadIdx.x >> 4][lane & 15] = acc[0];
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    float s = red[0][threadIdx.x];
#pragma unroll
    for (int r = 1; r < kBlock / kNnpChunk; ++r) s += red[r][threadIdx.x];
    part[(int64_t)(i0 + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

// phi_i = ke * (sum of the nbx partials of atom i, in order, FP64); one
// wavefront per NNP atom.  nbx = 0 (no MM atoms) gives phi = 0.
__global__ __launch_bounds__(kBlock) void k_mm_finish(const float* __restrict__ part, int nbx, int n,
                                                      DescParams p, float* __restrict__ x) {
  const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;   // wavefront-uniform
  double s = 0.0;
  for (int b = lane; b < nbx; b += 64) s += (double)part[(int64_t)i * nbx + b];
  s = wave_sum(s);
  if (lane == 0) x[(int64_t)i * p.stride + p.D] = (float)(p.ke * s);
}

// Adjoint: dE/dphi_i = g[i][D] (+ the predicted charge q_i of a network with
// a charge output, whose energy holds q_i phi_i);  dphi_i/dy_j = ke q_j f'(r) u,  f(r) = fc(r)/r,
// u = (y_j - x_i)/r.  MM atom j gets -sum_i dE/dphi_i dphi_i/dy_j (owned by
// its lane when one row covers every NNP atom, else FP64 atomics from each
// row, on distinct addresses); NNP atom i gets the opposite of its column
// sum, as per-workgroup partials part[(i * gridDim.x + blockIdx.x) * 3 + k].
__global__ __launch_bounds__(kBlock) void k_mm_bwd(const float4* __restrict__ spos, int n,
                                                   const float* __restrict__ mm_pos,
                                                   const float* __restrict__ mm_q, int n_mm,
                                                   const float* __restrict__ gx,
                                                   const float* __restrict__ qpred, DescParams p, Geometry g,
                                                   float* __restrict__ part,
                                                   double* __restrict__ mm_forces) {
  __shared__ float red[3][kBlock / kNnpChunk][kNnpChunk];   // [component][wavefront row][NNP atom]
  const int lane = threadIdx.x & 63;
  const int i0 = blockIdx.y * kNnpChunk, cnt = min(n - i0, kNnpChunk);
  const float rm2 = p.mm_cutoff * p.mm_cutoff;
  const float inv2rm = 0.5f / p.mm_cutoff;
  const float dfc_s = -0.5f * 3.14159265358979323846f / p.mm_cutoff;
  float ax[kNnpChunk], ay[kNnpChunk], az[kNnpChunk], ke_g[kNnpChunk];
#pragma unroll
  for (int c = 0; c < kNnpChunk; ++c) {
    ax[c] = ay[c] = az[c] = 0.f;
    ke_g[c] = 0.f;
    if (c < cnt) {
      const int i = i0 + c;
      float gi = gx[(int64_t)i * p.stride + p.D];
      if (qpred != nullptr) gi += qpred[i];
      ke_g[c] = (float)p.ke * gi;
    }
  }
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < n_mm; j += gridDim.x * kBlock) {
    const float yx = mm_pos[3 * (int64_t)j], yy = mm_pos[3 * (int64_t)j + 1], yz = mm_pos[3 * (int64_t)j + 2];
    const float q = mm_q[j];
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int c = 0; c < kNnpChunk; ++c) {
      if (c < cnt) {
        const float4 pi = spos[i0 + c];
        float dx, dy, dz, r2;
        mm_disp(pi, yx, yy, yz, g, dx, dy, dz, r2);
        if (r2 < rm2) {
          float ir = __builtin_amdgcn_rsqf(r2);
          float r = r2 * ir;
          float arg = r * inv2rm;
          float fc = 0.5f * __builtin_amdgcn_cosf(arg) + 0.5f;
          float dfc = dfc_s * __builtin_amdgcn_sinf(arg);
          float fp = (dfc - fc * ir) * ir;            // d/dr (fc / r)
          float w = ke_g[c] * q * fp * ir;   // times u = d / r
          const float vx = w * dx, vy = w * dy, vz = w * dz;
          ax[c] += vx; ay[c] += vy; az[c] += vz;
          fx -= vx; fy -= vy; fz -= vz;
        }
      }
    }
    if (mm_forces != nullptr) {
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
  row_sum16(ax, lane);
  row_sum16(ay, lane);
  row_sum16(az, lane);
  red[0][threadIdx.x >> 4][lane & 15] = ax[0];
  red[1][threadIdx.x >> 4][lane & 15] = ay[0];
  red[2][threadIdx.x >> 4][lane & 15] = az[0];
  __syncthreads();
  if ((int)threadIdx.x < 3 * cnt) {
    const int c = threadIdx.x / 3, k = threadIdx.x - 3 * c;
    float s = red[k][0][c];
#pragma unroll
    for (int r = 1; r < kBlock / kNnpChunk; ++r) s += red[k][r][c];
    part[((int64_t)(i0 + c) * gridDim.x + blockIdx.x) * 3 + k] = s;
  }
}

// NNP atom i: its partials summed in order (FP64) and added to its force
// row (or its link atom's); one wavefront per atom, so each row has one writer.
__global__ __launch_bounds__(kBlock) void k_mm_bwd_finish(const float* __restrict__ part, int nbx, int n,
                                                          const int* __restrict__ slot_atom,
                                                          double* __restrict__ forces,
                                                          double* __restrict__ link_forces) {
  const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;   // wavefront-uniform
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int b = lane; b < nbx; b += 64) {
    const float* v = part + ((int64_t)i * nbx + b) * 3;
    sx += (double)v[0]; sy += (double)v[1]; sz += (double)v[2];
  }
  sx = wave_sum(sx); sy = wave_sum(sy); sz = wave_sum(sz);
  if (lane == 0) {
    const int a = slot_atom[i];   // a < 0: link atom -1 - a
    double* f = a >= 0 ? forces + 3 * (int64_t)a : link_forces + 3 * (int64_t)(-1 - a);
    f[0] += sx; f[1] += sy; f[2] += sz;
  }
}

inline int mm_blocks(int n_mm) {
  const int b = (n_mm + kBlock - 1) / kBlock;
  return b < kMaxMmBlocks ? b : kMaxMmBlocks;
}

inline int wave_blocks(int n) { return (int)(((int64_t)n * 64 + kBlock - 1) / kBlock); }

}  // namespace

size_t mm_partial_floats(int max_atoms, int max_mm) {
  return max_mm > 0 ? 3 * (size_t)max_atoms * (size_t)mm_blocks(max_mm) : 0;
}

hipError_t launch_mm_fwd(nnp_model& m, int n, int n_mm, const float* mm_pos, const float* mm_q,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int nbx = n_mm > 0 ? mm_blocks(n_mm) : 0;
  if (nbx > 0) {
    if (m.d_mm_part == nullptr || (size_t)n * nbx > mm_partial_floats(m.max_atoms, m.max_mm))
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mm_fwd, dim3(nbx, (n + kNnpChunk - 1) / kNnpChunk), dim3(kBlock), 0, st, m.d_spos, n,
                       mm_pos, mm_q, n_mm, m.dp, m.geo, m.d_mm_part);
  }
  hipLaunchKernelGGL(k_mm_finish, dim3(wave_blocks(n)), dim3(kBlock), 0, st, m.d_mm_part, nbx, n, m.dp, m.d_x);
  return hipGetLastError();
}

hipError_t launch_mm_bwd(nnp_model& m, int n, int n_mm, const float* mm_pos, const float* mm_q,
                         double* forces, double* mm_forces, hipStream_t st) {
  if (n == 0 || n_mm == 0) return hipSuccess;
  const int nbx = mm_blocks(n_mm);
  if (m.d_mm_part == nullptr || 3 * (size_t)n * nbx > mm_partial_floats(m.max_atoms, m.max_mm))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mm_bwd, dim3(nbx, (n + kNnpChunk - 1) / kNnpChunk), dim3(kBlock), 0, st, m.d_spos, n,
                     mm_pos, mm_q, n_mm, m.d_g, m.charges ? m.d_q : nullptr, m.dp, m.geo, m.d_mm_part, mm_forces);
  hipLaunchKernelGGL(k_mm_bwd_finish, dim3(wave_blocks(n)), dim3(kBlock), 0, st, m.d_mm_part, nbx, n,
                     m.d_slot_atom, forces, m.d_link_F);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p, (int)n);
  return hipGetLastError();
}

}  // namespace nnp
