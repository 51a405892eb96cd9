// Symmetry-function descriptors (forward) and their adjoint (backward with
// the FP64 force scatter).
//
// Work decomposition: one lane per (atom, block), where a block is either the
// radial block of one neighbour species (16 outputs) or the angular block of
// one unordered species pair (8 x 4 outputs).  Consecutive lanes take
// consecutive atoms of the same block kind, so a wavefront runs one code
// path.  A lane keeps its outputs in registers and writes them once; no
// cross-lane reduction and no atomics are needed in the forward pass.
//
// Radial   G[s][k]   = sum_j exp(-eta_r (r - Rs_k)^2) fc(r; Rc)
// Angular  G[p][m][n] = 2^(1-zeta) sum_{j<k} (1 + cos(theta' - theta_n))^zeta
//                         exp(-eta_a (rbar - Ra_m)^2) fc(r_j; Rca) fc(r_k; Rca)
// with theta' = arccos(0.95 cos theta).  cos(theta' - theta_n) is expanded as
// cos theta' cos theta_n + sin theta' sin theta_n, where cos theta' = 0.95 c
// and sin theta' = sqrt(1 - (0.95 c)^2) >= 0.312, so no arccos is evaluated.
//
// Transcendentals use the hardware exp2 / log2 / sin / cos / sqrt / rsq
// instructions (arguments pre-scaled: exp(x) = exp2(x log2 e), cos(pi r/R) =
// cos of r/(2R) revolutions).
#include "nnp_internal.h"

namespace nnp {
namespace {

constexpr int kBlock = 256;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

struct Geo {
  float dx, dy, dz, r, ir;
};

__device__ __forceinline__ Geo displacement(const float4& pi, const float4& pj, const Geometry& g) {
  Geo o;
  float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
  if (g.periodic) {
    dx -= g.box[0] * rintf(dx * g.inv_box[0]);
    dy -= g.box[1] * rintf(dy * g.inv_box[1]);
    dz -= g.box[2] * rintf(dz * g.inv_box[2]);
  }
  float r2 = dx * dx + dy * dy + dz * dz;
  float ir = rsq(r2);
  o.dx = dx; o.dy = dy; o.dz = dz;
  o.r = r2 * ir;
  o.ir = ir;
  return o;
}

struct Consts {
  // pre-scaled constants
  float eta_r_l2, eta_a_l2;      // eta * log2(e)
  float inv2rc, inv2rca;         // 1 / (2 Rc): cos(pi r / Rc) = cos_rev(r / (2 Rc))
  float dfc_r, dfc_a;            // -0.5 pi / Rc
};

__device__ __forceinline__ Consts make_consts(const DescParams& p) {
  Consts c;
  c.eta_r_l2 = p.eta_rad * kLog2e;
  c.eta_a_l2 = p.eta_ang * kLog2e;
  c.inv2rc = 0.5f / p.rc_rad;
  c.inv2rca = 0.5f / p.rc_ang;
  c.dfc_r = -0.5f * 3.14159265358979323846f / p.rc_rad;
  c.dfc_a = -0.5f * 3.14159265358979323846f / p.rc_ang;
  return c;
}

struct DescArgs {
  const float4* spos;
  const int* slot_atom;
  const int* rad;
  const int* ang;
  const int* rad_off;
  const int* ang_off;
  int max_rad, max_ang;
  int n;
  float* x;         // forward output
  const float* g;   // backward input
  double* forces;   // backward output [atoms][3]
};

__global__ __launch_bounds__(kBlock) void k_desc_fwd(DescArgs a, DescParams p, Geometry geo) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  int blk = gid / a.n;
  int i = gid - blk * a.n;
  if (blk >= p.S + p.P) return;
  const Consts c = make_consts(p);
  const float4 pi = a.spos[i];
  const int S1 = p.S + 1;
  float* xo = a.x + (int64_t)i * p.stride;
  if (blk < p.S) {
    // radial block of neighbour species s = blk
    const int* row = a.rad + (int64_t)i * a.max_rad;
    int j0 = a.rad_off[(int64_t)i * S1 + blk], j1 = a.rad_off[(int64_t)i * S1 + blk + 1];
    float acc[kRadShifts];
#pragma unroll
    for (int k = 0; k < kRadShifts; ++k) acc[k] = 0.f;
    for (int jj = j0; jj < j1; ++jj) {
      Geo d = displacement(pi, a.spos[row[jj]], geo);
      float fc = 0.5f * cos_rev(d.r * c.inv2rc) + 0.5f;
#pragma unroll
      for (int k = 0; k < kRadShifts; ++k) {
        float t = d.r - p.rad_shift[k];
        acc[k] += ex2(-c.eta_r_l2 * t * t) * fc;
      }
    }
    float4* o4 = reinterpret_cast<float4*>(xo + blk * kRadShifts);
#pragma unroll
    for (int k = 0; k < kRadShifts / 4; ++k)
      o4[k] = make_float4(acc[4 * k], acc[4 * k + 1], acc[4 * k + 2], acc[4 * k + 3]);
    return;
  }
  // angular block of species pair q
  const int q = blk - p.S;
  const int sa = p.pair_a[q], sb = p.pair_b[q];
  const int* row = a.ang + (int64_t)i * a.max_ang;
  const int a0 = a.ang_off[(int64_t)i * S1 + sa], a1 = a.ang_off[(int64_t)i * S1 + sa + 1];
  const int b0 = a.ang_off[(int64_t)i * S1 + sb], b1 = a.ang_off[(int64_t)i * S1 + sb + 1];
  float acc[kAngShifts][kAngSects];
#pragma unroll
  for (int m = 0; m < kAngShifts; ++m)
#pragma unroll
    for (int n = 0; n < kAngSects; ++n) acc[m][n] = 0.f;
  for (int jj = a0; jj < a1; ++jj) {
    Geo dj = displacement(pi, a.spos[row[jj]], geo);
    float fcj = p.ang_pref * (0.5f * cos_rev(dj.r * c.inv2rca) + 0.5f);
    float ujx = dj.dx * dj.ir, ujy = dj.dy * dj.ir, ujz = dj.dz * dj.ir;
    for (int kk = (sa == sb ? jj + 1 : b0); kk < b1; ++kk) {
      Geo dk = displacement(pi, a.spos[row[kk]], geo);
      float fck = 0.5f * cos_rev(dk.r * c.inv2rca) + 0.5f;
      float cs = (ujx * dk.dx + ujy * dk.dy + ujz * dk.dz) * dk.ir;
      float ct = 0.95f * cs;
      float st = __builtin_amdgcn_sqrtf(1.f - ct * ct);
      float F = fcj * fck;
      float rbar = 0.5f * (dj.r + dk.r);
      float A[kAngSects];
#pragma unroll
      for (int n = 0; n < kAngSects; ++n) {
        float base = 1.f + ct * p.cos_sect[n] + st * p.sin_sect[n];
        A[n] = F * ex2(p.zeta * lg2(base));
      }
#pragma unroll
      for (int m = 0; m < kAngShifts; ++m) {
        float t = rbar - p.ang_shift[m];
        float B = ex2(-c.eta_a_l2 * t * t);
#pragma unroll
        for (int n = 0; n < kAngSects; ++n) acc[m][n] += B * A[n];
      }
    }
  }
  float4* o4 = reinterpret_cast<float4*>(xo + p.S * kRadShifts + q * kAngShifts * kAngSects);
#pragma unroll
  for (int m = 0; m < kAngShifts; ++m) o4[m] = make_float4(acc[m][0], acc[m][1], acc[m][2], acc[m][3]);
}

// Adjoint, one wavefront per centre atom i (no global atomics).
//
// E depends on d_ij = x_j - x_i, so a pair vector v = dE/d(d_ij) contributes
// -v to F_j and +v to F_i.  The wavefront
//   1. evaluates the radial terms, one neighbour per lane, storing v in an
//      FP64 LDS slot per radial neighbour;
//   2. caches the geometry of the angular neighbours in LDS;
//   3. evaluates the angular triplets (j < k), one per lane, adding v_j and
//      v_k into the neighbours' slots with FP64 LDS atomics;
//   4. hands each neighbour's total to that neighbour: the centre's position
//      in the neighbour's own list (lists are symmetric and sorted by slot
//      within each species segment) is found by binary search, and the
//      total, rounded once to FP32, is stored there -- each entry has exactly
//      one writer;
//   5. stores the centre's own total (FP64).
// k_force_gather then sums, per atom and in FP64, its own total and the
// entries of its list, and adds the result to the caller's force array.
struct BwdArgs {
  const float4* spos;
  const int* rad;
  const int* ang;
  const int* angpos;
  const int* rad_off;
  const int* ang_off;
  int max_rad, max_ang, n;
  const float* g;
  float4* contrib;   // [n][max_rad]
  double* self;      // [n][3]
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(64) void k_desc_bwd(BwdArgs a, DescParams p, Geometry geo) {
  extern __shared__ double smem_d[];
  double* slot = smem_d;                                          // [max_rad][3]
  float* gang = reinterpret_cast<float*>(slot + 3 * a.max_rad);   // [max_ang][8]
  int* rpos = reinterpret_cast<int*>(gang + 8 * a.max_ang);       // [max_ang]
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const Consts c = make_consts(p);
  const float4 pi = a.spos[i];
  const int S1 = p.S + 1;
  const int nr = a.rad_off[(int64_t)i * S1 + p.S];
  const int na = a.ang_off[(int64_t)i * S1 + p.S];
  const int* rrow = a.rad + (int64_t)i * a.max_rad;
  const int* arow = a.ang + (int64_t)i * a.max_ang;
  const float* gi = a.g + (int64_t)i * p.stride;
  double fx = 0.0, fy = 0.0, fz = 0.0;

  // 1. radial pairs
  for (int t = lane; t < nr; t += 64) {
    const float4 pj = a.spos[rrow[t]];
    const int sj = __float_as_int(pj.w);
    Geo d = displacement(pi, pj, geo);
    float arg = d.r * c.inv2rc;
    float fc = 0.5f * cos_rev(arg) + 0.5f;
    float dfc = c.dfc_r * sin_rev(arg);
    const float4* g4 = reinterpret_cast<const float4*>(gi + sj * kRadShifts);
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int q = 0; q < kRadShifts / 4; ++q) {
      float4 gv = g4[q];
      float gk[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float tt = d.r - p.rad_shift[4 * q + u];
        float B = gk[u] * ex2(-c.eta_r_l2 * tt * tt);
        s0 += B;
        s1 += B * tt;
      }
    }
    float dTdr = dfc * s0 - 2.f * p.eta_rad * fc * s1;
    float w = dTdr * d.ir;
    float vx = w * d.dx, vy = w * d.dy, vz = w * d.dz;
    slot[3 * t + 0] = vx;
    slot[3 * t + 1] = vy;
    slot[3 * t + 2] = vz;
    fx += vx; fy += vy; fz += vz;
  }
  // 2. angular neighbour geometry
  for (int u = lane; u < na; u += 64) {
    const float4 pj = a.spos[arow[u]];
    Geo d = displacement(pi, pj, geo);
    float arg = d.r * c.inv2rca;
    float* o = gang + 8 * u;
    o[0] = d.dx * d.ir; o[1] = d.dy * d.ir; o[2] = d.dz * d.ir;
    o[3] = d.r; o[4] = d.ir;
    o[5] = 0.5f * cos_rev(arg) + 0.5f;
    o[6] = c.dfc_a * sin_rev(arg);
    o[7] = pj.w;
    rpos[u] = a.angpos[(int64_t)i * a.max_ang + u];
  }
  __syncthreads();
  // 3. angular triplets, j < k in the angular list
  const int T = na * (na - 1) / 2;
  for (int t = lane; t < T; t += 64) {
    int b = (int)((1.f + __builtin_amdgcn_sqrtf(1.f + 8.f * (float)t)) * 0.5f);
    while (b * (b - 1) / 2 > t) --b;
    while ((b + 1) * b / 2 <= t) ++b;
    const int aj = t - b * (b - 1) / 2;
    const float* oj = gang + 8 * aj;
    const float* ok = gang + 8 * b;
    const float ujx = oj[0], ujy = oj[1], ujz = oj[2], rj = oj[3], irj = oj[4], fcj = oj[5], dfcj = oj[6];
    const float ukx = ok[0], uky = ok[1], ukz = ok[2], rk = ok[3], irk = ok[4], fck = ok[5], dfck = ok[6];
    const int sj = __float_as_int(oj[7]), sk = __float_as_int(ok[7]);
    const int q = p.class_of[sj][sk];
    const float4* g4 = reinterpret_cast<const float4*>(gi + p.S * kRadShifts + q * kAngShifts * kAngSects);
    float cs = ujx * ukx + ujy * uky + ujz * ukz;
    float ct = 0.95f * cs;
    float st = __builtin_amdgcn_sqrtf(1.f - ct * ct);
    float ist = __builtin_amdgcn_rcpf(st);
    float rbar = 0.5f * (rj + rk);
    float A[kAngSects], dA[kAngSects];
#pragma unroll
    for (int n = 0; n < kAngSects; ++n) {
      float base = 1.f + ct * p.cos_sect[n] + st * p.sin_sect[n];
      float An = ex2(p.zeta * lg2(base));
      A[n] = An;
      dA[n] = p.zeta * An * __builtin_amdgcn_rcpf(base) * 0.95f * (p.cos_sect[n] - ct * ist * p.sin_sect[n]);
    }
    float h[kAngSects] = {0.f, 0.f, 0.f, 0.f};
    float sdr = 0.f;
#pragma unroll
    for (int m = 0; m < kAngShifts; ++m) {
      float4 gv = g4[m];
      float G[4] = {gv.x, gv.y, gv.z, gv.w};
      float tt = rbar - p.ang_shift[m];
      float B = ex2(-c.eta_a_l2 * tt * tt);
      float km = 0.f;
#pragma unroll
      for (int n = 0; n < kAngSects; ++n) {
        h[n] += G[n] * B;
        km += G[n] * A[n];
      }
      sdr += -2.f * p.eta_ang * tt * B * km;
    }
    float SA = 0.f, SdA = 0.f;
#pragma unroll
    for (int n = 0; n < kAngSects; ++n) {
      SA += h[n] * A[n];
      SdA += h[n] * dA[n];
    }
    float F = p.ang_pref * fcj * fck;
    float dTdc = F * SdA;
    float dTdrbar = F * sdr;
    float dTdrj = 0.5f * dTdrbar + p.ang_pref * dfcj * fck * SA;
    float dTdrk = 0.5f * dTdrbar + p.ang_pref * fcj * dfck * SA;
    float cj = dTdc * irj, ck = dTdc * irk;
    float vjx = cj * (ukx - cs * ujx) + dTdrj * ujx;
    float vjy = cj * (uky - cs * ujy) + dTdrj * ujy;
    float vjz = cj * (ukz - cs * ujz) + dTdrj * ujz;
    float vkx = ck * (ujx - cs * ukx) + dTdrk * ukx;
    float vky = ck * (ujy - cs * uky) + dTdrk * uky;
    float vkz = ck * (ujz - cs * ukz) + dTdrk * ukz;
    double* sjp = slot + 3 * rpos[aj];
    double* skp = slot + 3 * rpos[b];
    unsafeAtomicAdd(sjp + 0, (double)vjx);
    unsafeAtomicAdd(sjp + 1, (double)vjy);
    unsafeAtomicAdd(sjp + 2, (double)vjz);
    unsafeAtomicAdd(skp + 0, (double)vkx);
    unsafeAtomicAdd(skp + 1, (double)vky);
    unsafeAtomicAdd(skp + 2, (double)vkz);
    fx += (double)vjx + (double)vkx;
    fy += (double)vjy + (double)vky;
    fz += (double)vjz + (double)vkz;
  }
  __syncthreads();
  // 4. each neighbour's total goes to the centre's slot in the neighbour's list
  const int si = __float_as_int(pi.w);
  for (int t = lane; t < nr; t += 64) {
    const int j = rrow[t];
    const int* jrow = a.rad + (int64_t)j * a.max_rad;
    int lo = a.rad_off[(int64_t)j * S1 + si], hi = a.rad_off[(int64_t)j * S1 + si + 1] - 1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (jrow[mid] < i) lo = mid + 1; else hi = mid;
    }
    if (lo <= hi && jrow[lo] == i)
      a.contrib[(int64_t)j * a.max_rad + lo] =
          make_float4((float)-slot[3 * t], (float)-slot[3 * t + 1], (float)-slot[3 * t + 2], 0.f);
  }
  // 5. the centre's own total
  fx = wave_sum_d(fx);
  fy = wave_sum_d(fy);
  fz = wave_sum_d(fz);
  if (lane == 0) {
    a.self[3 * (int64_t)i + 0] = fx;
    a.self[3 * (int64_t)i + 1] = fy;
    a.self[3 * (int64_t)i + 2] = fz;
  }
}

// F_atom += self + sum over the atom's radial list entries (FP64), one thread per atom.
__global__ __launch_bounds__(kBlock) void k_force_gather(const float4* __restrict__ contrib,
                                                         const double* __restrict__ self,
                                                         const int* __restrict__ rad_off,
                                                         const int* __restrict__ slot_atom, int n, int S,
                                                         int max_rad, double* __restrict__ forces) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int nr = rad_off[(int64_t)i * (S + 1) + S];
  double fx = self[3 * (int64_t)i], fy = self[3 * (int64_t)i + 1], fz = self[3 * (int64_t)i + 2];
  const float4* row = contrib + (int64_t)i * max_rad;
  for (int t = 0; t < nr; ++t) {
    float4 v = row[t];
    fx += v.x; fy += v.y; fz += v.z;
  }
  double* f = forces + 3 * (int64_t)slot_atom[i];
  f[0] += fx;
  f[1] += fy;
  f[2] += fz;
}

DescArgs make_args(nnp_model& m, int n) {
  DescArgs a;
  a.spos = m.d_spos;
  a.slot_atom = m.d_slot_atom;
  a.rad = m.d_nbr_rad;
  a.ang = m.d_nbr_ang;
  a.rad_off = m.d_rad_off;
  a.ang_off = m.d_ang_off;
  a.max_rad = m.max_rad;
  a.max_ang = m.max_ang;
  a.n = n;
  a.x = m.d_x;
  a.g = m.d_g;
  a.forces = nullptr;
  return a;
}

}  // namespace

hipError_t launch_descriptor_fwd(nnp_model& m, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  DescArgs a = make_args(m, n);
  int64_t lanes = (int64_t)(m.S + m.P) * n;
  hipLaunchKernelGGL(k_desc_fwd, dim3((unsigned)((lanes + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     a, m.dp, m.geo);
  return hipGetLastError();
}

hipError_t launch_descriptor_bwd(nnp_model& m, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  BwdArgs a;
  a.spos = m.d_spos;
  a.rad = m.d_nbr_rad;
  a.ang = m.d_nbr_ang;
  a.angpos = m.d_angpos;
  a.rad_off = m.d_rad_off;
  a.ang_off = m.d_ang_off;
  a.max_rad = m.max_rad;
  a.max_ang = m.max_ang;
  a.n = n;
  a.g = m.d_g;
  a.contrib = m.d_contrib;
  a.self = m.d_self;
  size_t lds = sizeof(double) * 3 * (size_t)m.max_rad + sizeof(float) * 8 * (size_t)m.max_ang +
               sizeof(int) * (size_t)m.max_ang;
  hipLaunchKernelGGL(k_desc_bwd, dim3(n), dim3(64), lds, st, a, m.dp, m.geo);
  return hipGetLastError();
}

hipError_t launch_force_gather(nnp_model& m, int n, double* forces, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_force_gather, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, m.d_contrib, m.d_self,
                     m.d_rad_off, m.d_slot_atom, n, m.S, m.max_rad, forces);
  return hipGetLastError();
}

}  // namespace nnp
