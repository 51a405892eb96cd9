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

__device__ __forceinline__ void add_force(double* f, int atom, double x, double y, double z) {
  double* p = f + 3 * (int64_t)atom;
  unsafeAtomicAdd(p + 0, x);
  unsafeAtomicAdd(p + 1, y);
  unsafeAtomicAdd(p + 2, z);
}

// Adjoint: g = dE/dx per atom -> dE/d(d_ij) per neighbour pair -> forces.
// E depends on d_ij = x_j - x_i, so a pair vector v = dE/d(d_ij) gives
// F_j -= v and F_i += v.  The centre's total and each outer neighbour's total
// are accumulated in FP64 registers before one atomic add; inner neighbours
// of the angular double loop are added per pair.
__global__ __launch_bounds__(kBlock) void k_desc_bwd(DescArgs a, DescParams p, Geometry geo) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  int blk = gid / a.n;
  int i = gid - blk * a.n;
  if (blk >= p.S + p.P) return;
  const Consts c = make_consts(p);
  const float4 pi = a.spos[i];
  const int S1 = p.S + 1;
  const float* gi = a.g + (int64_t)i * p.stride;
  double fix = 0.0, fiy = 0.0, fiz = 0.0;
  if (blk < p.S) {
    const int* row = a.rad + (int64_t)i * a.max_rad;
    int j0 = a.rad_off[(int64_t)i * S1 + blk], j1 = a.rad_off[(int64_t)i * S1 + blk + 1];
    float gk[kRadShifts];
    const float4* g4 = reinterpret_cast<const float4*>(gi + blk * kRadShifts);
#pragma unroll
    for (int k = 0; k < kRadShifts / 4; ++k) {
      float4 v = g4[k];
      gk[4 * k] = v.x; gk[4 * k + 1] = v.y; gk[4 * k + 2] = v.z; gk[4 * k + 3] = v.w;
    }
    for (int jj = j0; jj < j1; ++jj) {
      int j = row[jj];
      Geo d = displacement(pi, a.spos[j], geo);
      float arg = d.r * c.inv2rc;
      float fc = 0.5f * cos_rev(arg) + 0.5f;
      float dfc = c.dfc_r * sin_rev(arg);
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int k = 0; k < kRadShifts; ++k) {
        float t = d.r - p.rad_shift[k];
        float B = gk[k] * ex2(-c.eta_r_l2 * t * t);
        s0 += B;
        s1 += B * t;
      }
      float dTdr = dfc * s0 - 2.f * p.eta_rad * fc * s1;
      float w = dTdr * d.ir;
      float vx = w * d.dx, vy = w * d.dy, vz = w * d.dz;
      add_force(a.forces, a.slot_atom[j], -(double)vx, -(double)vy, -(double)vz);
      fix += vx; fiy += vy; fiz += vz;
    }
    add_force(a.forces, a.slot_atom[i], fix, fiy, fiz);
    return;
  }
  const int q = blk - p.S;
  const int sa = p.pair_a[q], sb = p.pair_b[q];
  const int* row = a.ang + (int64_t)i * a.max_ang;
  const int a0 = a.ang_off[(int64_t)i * S1 + sa], a1 = a.ang_off[(int64_t)i * S1 + sa + 1];
  const int b0 = a.ang_off[(int64_t)i * S1 + sb], b1 = a.ang_off[(int64_t)i * S1 + sb + 1];
  float G[kAngShifts][kAngSects];
  const float4* g4 = reinterpret_cast<const float4*>(gi + p.S * kRadShifts + q * kAngShifts * kAngSects);
#pragma unroll
  for (int m = 0; m < kAngShifts; ++m) {
    float4 v = g4[m];
    G[m][0] = v.x; G[m][1] = v.y; G[m][2] = v.z; G[m][3] = v.w;
  }
  for (int jj = a0; jj < a1; ++jj) {
    int j = row[jj];
    Geo dj = displacement(pi, a.spos[j], geo);
    float argj = dj.r * c.inv2rca;
    float fcj = 0.5f * cos_rev(argj) + 0.5f;
    float dfcj = c.dfc_a * sin_rev(argj);
    float ujx = dj.dx * dj.ir, ujy = dj.dy * dj.ir, ujz = dj.dz * dj.ir;
    double fjx = 0.0, fjy = 0.0, fjz = 0.0;
    for (int kk = (sa == sb ? jj + 1 : b0); kk < b1; ++kk) {
      int k = row[kk];
      Geo dk = displacement(pi, a.spos[k], geo);
      float argk = dk.r * c.inv2rca;
      float fck = 0.5f * cos_rev(argk) + 0.5f;
      float dfck = c.dfc_a * sin_rev(argk);
      float ukx = dk.dx * dk.ir, uky = dk.dy * dk.ir, ukz = dk.dz * dk.ir;
      float cs = ujx * ukx + ujy * uky + ujz * ukz;
      float ct = 0.95f * cs;
      float st = __builtin_amdgcn_sqrtf(1.f - ct * ct);
      float ist = __builtin_amdgcn_rcpf(st);
      float rbar = 0.5f * (dj.r + dk.r);
      float A[kAngSects], dA[kAngSects];
#pragma unroll
      for (int n = 0; n < kAngSects; ++n) {
        float base = 1.f + ct * p.cos_sect[n] + st * p.sin_sect[n];
        float An = ex2(p.zeta * lg2(base));
        A[n] = An;
        // d/dc of (1 + cos(theta' - theta_n))^zeta
        dA[n] = p.zeta * An * __builtin_amdgcn_rcpf(base) * 0.95f * (p.cos_sect[n] - ct * ist * p.sin_sect[n]);
      }
      float h[kAngSects] = {0.f, 0.f, 0.f, 0.f};
      float sdr = 0.f;   // sum_m dB_m/drbar * sum_n G[m][n] A_n
#pragma unroll
      for (int m = 0; m < kAngShifts; ++m) {
        float t = rbar - p.ang_shift[m];
        float B = ex2(-c.eta_a_l2 * t * t);
        float km = 0.f;
#pragma unroll
        for (int n = 0; n < kAngSects; ++n) {
          h[n] += G[m][n] * B;
          km += G[m][n] * A[n];
        }
        sdr += -2.f * p.eta_ang * t * B * km;
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
      float cj = dTdc * dj.ir, ck = dTdc * dk.ir;
      float vjx = cj * (ukx - cs * ujx) + dTdrj * ujx;
      float vjy = cj * (uky - cs * ujy) + dTdrj * ujy;
      float vjz = cj * (ukz - cs * ujz) + dTdrj * ujz;
      float vkx = ck * (ujx - cs * ukx) + dTdrk * ukx;
      float vky = ck * (ujy - cs * uky) + dTdrk * uky;
      float vkz = ck * (ujz - cs * ukz) + dTdrk * ukz;
      add_force(a.forces, a.slot_atom[k], -(double)vkx, -(double)vky, -(double)vkz);
      fjx += vjx; fjy += vjy; fjz += vjz;
      fix += (double)vjx + (double)vkx;
      fiy += (double)vjy + (double)vky;
      fiz += (double)vjz + (double)vkz;
    }
    if (fjx != 0.0 || fjy != 0.0 || fjz != 0.0) add_force(a.forces, a.slot_atom[j], -fjx, -fjy, -fjz);
  }
  add_force(a.forces, a.slot_atom[i], fix, fiy, fiz);
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

hipError_t launch_descriptor_bwd(nnp_model& m, int n, double* forces, hipStream_t st) {
  if (n == 0) return hipSuccess;
  DescArgs a = make_args(m, n);
  a.forces = forces;
  int64_t lanes = (int64_t)(m.S + m.P) * n;
  hipLaunchKernelGGL(k_desc_bwd, dim3((unsigned)((lanes + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     a, m.dp, m.geo);
  return hipGetLastError();
}

}  // namespace nnp
