// Symmetry-function descriptors (forward) and their adjoint (backward with
// the FP64 force scatter).
//
// Both passes run one wavefront per atom.  An output block is either the
// radial block of one neighbour species (16 outputs) or the angular block of
// one unordered species pair (8 x 4 outputs).
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

// Split the 64 lanes of a wavefront over nb output blocks in proportion to
// their work counts (every block with work gets at least one lane), and
// return this lane's block, its rank in the block and the block's lane count.
__device__ __forceinline__ void split_lanes(const int* cnt, int nb, int lane, int* my_b, int* my_rank, int* my_len,
                                            int* start, int* len) {
  int total = 0;
  for (int b = 0; b < nb; ++b) total += cnt[b];
  const float scale = total > 0 ? 64.f / (float)total : 0.f;
  int used = 0;
  for (int b = 0; b < nb; ++b) {
    len[b] = cnt[b] > 0 ? max(1, (int)((float)cnt[b] * scale)) : 0;
    used += len[b];
  }
  while (used > 64) {  // only when many tiny blocks were rounded up to one lane
    int k = 0;
    for (int b = 1; b < nb; ++b) if (len[b] > len[k]) k = b;
    --len[k];
    --used;
  }
  while (used < 64 && total > 0) {  // spare lanes go to the block with most work per lane
    int k = -1;
    for (int b = 0; b < nb; ++b)
      if (cnt[b] > 0 && (k < 0 || cnt[b] * len[k] > cnt[k] * len[b])) k = b;
    ++len[k];
    ++used;
  }
  int run = 0;
  *my_b = -1;
  *my_rank = 0;
  *my_len = 0;
  for (int b = 0; b < nb; ++b) {
    start[b] = run;
    if (lane >= run && lane < run + len[b]) {
      *my_b = b;
      *my_rank = lane - run;
      *my_len = len[b];
    }
    run += len[b];
  }
}

// Forward descriptors, one wavefront per atom.  Radial phase: the lanes are
// split over the S neighbour-species segments of the radial list, each lane
// accumulating the 16 radial terms of its neighbours in registers.  Angular
// phase: the angular neighbours' geometry is cached in LDS (one array per
// component) and the lanes are split over the P species-pair classes; each
// lane takes a contiguous range of its class's (j, k) pairs, walked without
// divisions, and accumulates the 32 terms in registers.  Each phase ends
// with a fixed-order reduction of the per-lane partial sums through LDS.
struct FwdArgs {
  const float4* spos;
  const int* rad;
  const int* ang;
  const int* rad_off;
  const int* ang_off;
  int max_rad, max_ang, n;
  float* x;
};

constexpr int kPartStride = 33;  // padded row of the per-lane partial sums

__global__ __launch_bounds__(64) void k_desc_fwd(FwdArgs a, DescParams p, Geometry geo) {
  extern __shared__ float smem_f[];
  float* part = smem_f;                      // [64][kPartStride]
  float* gux = part + 64 * kPartStride;      // angular neighbours, one array per component
  float* guy = gux + a.max_ang;
  float* guz = guy + a.max_ang;
  float* gr = guz + a.max_ang;
  float* gfc = gr + a.max_ang;
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const Consts c = make_consts(p);
  const float4 pi = a.spos[i];
  const int S1 = p.S + 1;
  const int* roff = a.rad_off + (int64_t)i * S1;
  const int* aoff = a.ang_off + (int64_t)i * S1;
  const int* rrow = a.rad + (int64_t)i * a.max_rad;
  const int* arow = a.ang + (int64_t)i * a.max_ang;
  float* xo = a.x + (int64_t)i * p.stride;
  int cnt[kMaxPairs], st[kMaxPairs], len[kMaxPairs];
  int my_b, my_rank, my_len;

  // ---- radial phase
  for (int s = 0; s < p.S; ++s) cnt[s] = roff[s + 1] - roff[s];
  split_lanes(cnt, p.S, lane, &my_b, &my_rank, &my_len, st, len);
  {
    float acc[kRadShifts];
#pragma unroll
    for (int k = 0; k < kRadShifts; ++k) acc[k] = 0.f;
    if (my_b >= 0) {
      const int t1 = roff[my_b + 1];
      for (int t = roff[my_b] + my_rank; t < t1; t += my_len) {
        Geo d = displacement(pi, a.spos[rrow[t]], geo);
        float fc = 0.5f * cos_rev(d.r * c.inv2rc) + 0.5f;
#pragma unroll
        for (int k = 0; k < kRadShifts; ++k) {
          float tt = d.r - p.rad_shift[k];
          acc[k] += ex2(-c.eta_r_l2 * tt * tt) * fc;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kRadShifts; ++k) part[lane * kPartStride + k] = acc[k];
  }
  // angular neighbour geometry
  const int na = aoff[p.S];
  for (int u = lane; u < na; u += 64) {
    Geo d = displacement(pi, a.spos[arow[u]], geo);
    gux[u] = d.dx * d.ir;
    guy[u] = d.dy * d.ir;
    guz[u] = d.dz * d.ir;
    gr[u] = d.r;
    gfc[u] = 0.5f * cos_rev(d.r * c.inv2rca) + 0.5f;
  }
  __syncthreads();
  for (int o = lane; o < p.S * kRadShifts; o += 64) {
    const int b = o / kRadShifts, k = o % kRadShifts;
    float v = 0.f;
    for (int l = st[b]; l < st[b] + len[b]; ++l) v += part[l * kPartStride + k];
    xo[o] = v;
  }
  __syncthreads();

  // ---- angular phase
  for (int q = 0; q < p.P; ++q) {
    const int na_ = aoff[p.pair_a[q] + 1] - aoff[p.pair_a[q]];
    const int nb_ = aoff[p.pair_b[q] + 1] - aoff[p.pair_b[q]];
    cnt[q] = p.pair_a[q] == p.pair_b[q] ? na_ * (na_ - 1) / 2 : na_ * nb_;
  }
  split_lanes(cnt, p.P, lane, &my_b, &my_rank, &my_len, st, len);
  {
    float acc[kAngShifts][kAngSects];
#pragma unroll
    for (int m = 0; m < kAngShifts; ++m)
#pragma unroll
      for (int n = 0; n < kAngSects; ++n) acc[m][n] = 0.f;
    if (my_b >= 0) {
      const int sa = p.pair_a[my_b], sb = p.pair_b[my_b];
      const int oa = aoff[sa], ob = aoff[sb];
      const int nB = aoff[sb + 1] - ob;
      const int T = cnt[my_b];
      // contiguous range [r0, r1) of this lane
      const int r0 = (int)(((int64_t)T * my_rank) / my_len);
      const int r1 = (int)(((int64_t)T * (my_rank + 1)) / my_len);
      int uj, uk;      // same pair (j, k): walk k = 1..n-1, j = 0..k-1 (k-major)
      if (sa == sb) {
        int kk = (int)((1.f + __builtin_amdgcn_sqrtf(1.f + 8.f * (float)r0)) * 0.5f);
        while (kk * (kk - 1) / 2 > r0) --kk;
        while ((kk + 1) * kk / 2 <= r0) ++kk;
        uj = r0 - kk * (kk - 1) / 2;
        uk = kk;
      } else {         // different species: j-major over (j, k)
        uj = r0 / max(nB, 1);
        uk = r0 - uj * nB;
      }
      for (int r = r0; r < r1; ++r) {
        const int gj = oa + uj;
        const int gk = (sa == sb ? oa : ob) + uk;
        float cs = gux[gj] * gux[gk] + guy[gj] * guy[gk] + guz[gj] * guz[gk];
        float ct = 0.95f * cs;
        float sn = __builtin_amdgcn_sqrtf(1.f - ct * ct);
        float F = p.ang_pref * gfc[gj] * gfc[gk];
        float rbar = 0.5f * (gr[gj] + gr[gk]);
        float A[kAngSects];
#pragma unroll
        for (int n = 0; n < kAngSects; ++n) {
          float base = 1.f + ct * p.cos_sect[n] + sn * p.sin_sect[n];
          A[n] = F * ex2(p.zeta * lg2(base));
        }
#pragma unroll
        for (int m = 0; m < kAngShifts; ++m) {
          float tt = rbar - p.ang_shift[m];
          float B = ex2(-c.eta_a_l2 * tt * tt);
#pragma unroll
          for (int n = 0; n < kAngSects; ++n) acc[m][n] += B * A[n];
        }
        if (sa == sb) {
          if (++uj == uk) { uj = 0; ++uk; }
        } else {
          if (++uk == nB) { uk = 0; ++uj; }
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kAngShifts; ++m)
#pragma unroll
      for (int n = 0; n < kAngSects; ++n) part[lane * kPartStride + m * kAngSects + n] = acc[m][n];
  }
  __syncthreads();
  const int nang = p.P * kAngShifts * kAngSects;
  for (int o = lane; o < nang; o += 64) {
    const int q = o / (kAngShifts * kAngSects), e = o % (kAngShifts * kAngSects);
    float v = 0.f;
    for (int l = st[q]; l < st[q] + len[q]; ++l) v += part[l * kPartStride + e];
    xo[p.S * kRadShifts + o] = v;
  }
}

// Adjoint, one wavefront per centre atom i (no global atomics).
//
// E depends on d_ij = x_j - x_i, so a pair vector v = dE/d(d_ij) contributes
// -v to F_j and +v to F_i.  The wavefront
//   1. stages the centre's dE/dx row in LDS;
//   2. evaluates the radial terms, one neighbour per lane, storing v in an
//      FP64 LDS slot per radial neighbour;
//   3. caches the geometry of the angular neighbours in LDS;
//   4. evaluates the angular triplets (j < k, k-major), each lane walking a
//      contiguous range: v_j goes to j's slot with an FP64 LDS atomic add,
//      v_k is summed in registers while k stays the same;
//   5. hands each neighbour's total to that neighbour: the centre's position
//      in the neighbour's own list (lists are symmetric and sorted by slot
//      within each species segment) is found by binary search, and the
//      total, rounded once to FP32, is stored there -- each entry has exactly
//      one writer;
//   6. stores the centre's own total (FP64).
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
  double* sx = smem_d;                          // per radial neighbour, FP64
  double* sy = sx + a.max_rad;
  double* sz = sy + a.max_rad;
  float* gl = reinterpret_cast<float*>(sz + a.max_rad);   // [stride] dE/dx of the centre
  float* gux = gl + p.stride;                    // angular neighbours, one array per component
  float* guy = gux + a.max_ang;
  float* guz = guy + a.max_ang;
  float* gr = guz + a.max_ang;
  float* gir = gr + a.max_ang;
  float* gfc = gir + a.max_ang;
  float* gdfc = gfc + a.max_ang;
  int* gsp = reinterpret_cast<int*>(gdfc + a.max_ang);
  int* rpos = gsp + a.max_ang;
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const Consts c = make_consts(p);
  const float4 pi = a.spos[i];
  const int S1 = p.S + 1;
  const int nr = a.rad_off[(int64_t)i * S1 + p.S];
  const int na = a.ang_off[(int64_t)i * S1 + p.S];
  const int* rrow = a.rad + (int64_t)i * a.max_rad;
  const int* arow = a.ang + (int64_t)i * a.max_ang;
  double fx = 0.0, fy = 0.0, fz = 0.0;

  // 1. dE/dx row
  {
    const float4* g4 = reinterpret_cast<const float4*>(a.g + (int64_t)i * p.stride);
    float4* l4 = reinterpret_cast<float4*>(gl);
    for (int q = lane; q < p.D / 4; q += 64) l4[q] = g4[q];
  }
  // 3. angular neighbour geometry (before the barrier, together with 1.)
  for (int u = lane; u < na; u += 64) {
    const float4 pj = a.spos[arow[u]];
    Geo d = displacement(pi, pj, geo);
    float arg = d.r * c.inv2rca;
    gux[u] = d.dx * d.ir;
    guy[u] = d.dy * d.ir;
    guz[u] = d.dz * d.ir;
    gr[u] = d.r;
    gir[u] = d.ir;
    gfc[u] = 0.5f * cos_rev(arg) + 0.5f;
    gdfc[u] = c.dfc_a * sin_rev(arg);
    gsp[u] = __float_as_int(pj.w);
    rpos[u] = a.angpos[(int64_t)i * a.max_ang + u];
  }
  __syncthreads();
  // 2. radial pairs
  for (int t = lane; t < nr; t += 64) {
    const float4 pj = a.spos[rrow[t]];
    const int sj = __float_as_int(pj.w);
    Geo d = displacement(pi, pj, geo);
    float arg = d.r * c.inv2rc;
    float fc = 0.5f * cos_rev(arg) + 0.5f;
    float dfc = c.dfc_r * sin_rev(arg);
    const float4* g4 = reinterpret_cast<const float4*>(gl + sj * kRadShifts);
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
    sx[t] = vx;
    sy[t] = vy;
    sz[t] = vz;
    fx += vx; fy += vy; fz += vz;
  }
  __syncthreads();
  // 4. angular triplets (j < k, k-major), a contiguous range per lane
  const int T = na * (na - 1) / 2;
  const int r0 = (int)(((int64_t)T * lane) >> 6);
  const int r1 = (int)(((int64_t)T * (lane + 1)) >> 6);
  if (r0 < r1) {
    int k = (int)((1.f + __builtin_amdgcn_sqrtf(1.f + 8.f * (float)r0)) * 0.5f);
    while (k * (k - 1) / 2 > r0) --k;
    while ((k + 1) * k / 2 <= r0) ++k;
    int j = r0 - k * (k - 1) / 2;
    double kx = 0.0, ky = 0.0, kz = 0.0;   // running total of the current k
    for (int r = r0; r < r1; ++r) {
      const float ujx = gux[j], ujy = guy[j], ujz = guz[j], rj = gr[j], irj = gir[j], fcj = gfc[j], dfcj = gdfc[j];
      const float ukx = gux[k], uky = guy[k], ukz = guz[k], rk = gr[k], irk = gir[k], fck = gfc[k], dfck = gdfc[k];
      const int q = p.class_of[gsp[j]][gsp[k]];
      const float4* g4 = reinterpret_cast<const float4*>(gl + p.S * kRadShifts + q * kAngShifts * kAngSects);
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
      const int pj = rpos[j];
      unsafeAtomicAdd(sx + pj, (double)vjx);
      unsafeAtomicAdd(sy + pj, (double)vjy);
      unsafeAtomicAdd(sz + pj, (double)vjz);
      kx += vkx; ky += vky; kz += vkz;
      fx += (double)vjx + (double)vkx;
      fy += (double)vjy + (double)vky;
      fz += (double)vjz + (double)vkz;
      if (++j == k || r + 1 == r1) {   // k changes (or the range ends): flush its total
        const int pk = rpos[k];
        unsafeAtomicAdd(sx + pk, kx);
        unsafeAtomicAdd(sy + pk, ky);
        unsafeAtomicAdd(sz + pk, kz);
        kx = ky = kz = 0.0;
        if (j == k) { j = 0; ++k; }
      }
    }
  }
  __syncthreads();
  // 5. each neighbour's total goes to the centre's slot in the neighbour's list
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
      a.contrib[(int64_t)j * a.max_rad + lo] = make_float4((float)-sx[t], (float)-sy[t], (float)-sz[t], 0.f);
  }
  // 6. the centre's own total
  fx = wave_sum_d(fx);
  fy = wave_sum_d(fy);
  fz = wave_sum_d(fz);
  if (lane == 0) {
    a.self[3 * (int64_t)i + 0] = fx;
    a.self[3 * (int64_t)i + 1] = fy;
    a.self[3 * (int64_t)i + 2] = fz;
  }
}

// F_atom += self + sum over the atom's radial list entries (FP64): 16 lanes
// per atom, each summing a strided part of the row, then a shuffle tree.
__global__ __launch_bounds__(kBlock) void k_force_gather(const float4* __restrict__ contrib,
                                                         const double* __restrict__ self,
                                                         const int* __restrict__ rad_off,
                                                         const int* __restrict__ slot_atom, int n, int S,
                                                         int max_rad, double* __restrict__ forces,
                                                         double* __restrict__ link_forces) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid >> 4;
  const int sub = gid & 15;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (i < n) {
    const int nr = rad_off[(int64_t)i * (S + 1) + S];
    const float4* row = contrib + (int64_t)i * max_rad;
    for (int t = sub; t < nr; t += 16) {
      float4 v = row[t];
      fx += v.x; fy += v.y; fz += v.z;
    }
  }
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) {
    fx += __shfl_xor(fx, off, 64);
    fy += __shfl_xor(fy, off, 64);
    fz += __shfl_xor(fz, off, 64);
  }
  if (i < n && sub == 0) {
    const int a = slot_atom[i];   // a < 0: link atom -1 - a
    double* f = a >= 0 ? forces + 3 * (int64_t)a : link_forces + 3 * (int64_t)(-1 - a);
    f[0] += fx + self[3 * (int64_t)i];
    f[1] += fy + self[3 * (int64_t)i + 1];
    f[2] += fz + self[3 * (int64_t)i + 2];
  }
}

// Chain rule for link atoms (eq. 4): r_L = r_ML + d u/|u|, u = r_MM - r_ML, so
// F_MM += (d/|u|)(F_L - (F_L.u^) u^) and F_ML += F_L - (d/|u|)(F_L - (F_L.u^) u^).
// FP64 atomics: an ML atom may carry several links.
__global__ __launch_bounds__(kBlock) void k_link_redistribute(const double* __restrict__ link_forces,
                                                              const int* __restrict__ ml, const int* __restrict__ mm,
                                                              int n_links, float d, const float* __restrict__ pos,
                                                              Geometry g, double* __restrict__ forces) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_links) return;
  const int a = ml[l], b = mm[l];
  double ux = (double)pos[3 * (int64_t)b] - pos[3 * (int64_t)a];
  double uy = (double)pos[3 * (int64_t)b + 1] - pos[3 * (int64_t)a + 1];
  double uz = (double)pos[3 * (int64_t)b + 2] - pos[3 * (int64_t)a + 2];
  if (g.periodic) {
    ux -= g.box[0] * rint(ux / g.box[0]);
    uy -= g.box[1] * rint(uy / g.box[1]);
    uz -= g.box[2] * rint(uz / g.box[2]);
  }
  const double inv = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
  ux *= inv; uy *= inv; uz *= inv;
  const double fx = link_forces[3 * l], fy = link_forces[3 * l + 1], fz = link_forces[3 * l + 2];
  const double s = (double)d * inv;
  const double fu = fx * ux + fy * uy + fz * uz;
  const double px = s * (fx - fu * ux), py = s * (fy - fu * uy), pz = s * (fz - fu * uz);
  unsafeAtomicAdd(forces + 3 * (int64_t)b + 0, px);
  unsafeAtomicAdd(forces + 3 * (int64_t)b + 1, py);
  unsafeAtomicAdd(forces + 3 * (int64_t)b + 2, pz);
  unsafeAtomicAdd(forces + 3 * (int64_t)a + 0, fx - px);
  unsafeAtomicAdd(forces + 3 * (int64_t)a + 1, fy - py);
  unsafeAtomicAdd(forces + 3 * (int64_t)a + 2, fz - pz);
}

}  // namespace

hipError_t launch_link_redistribute(nnp_model& m, const float* pos, double* forces, hipStream_t st) {
  if (m.n_links_dev == 0) return hipSuccess;
  hipLaunchKernelGGL(k_link_redistribute, dim3((m.n_links_dev + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                     m.d_link_F, m.d_link_ml, m.d_link_mm, m.n_links_dev, m.link_d, pos, m.geo, forces);
  return hipGetLastError();
}

hipError_t launch_descriptor_fwd(nnp_model& m, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  FwdArgs a;
  a.spos = m.d_spos;
  a.rad = m.d_nbr_rad;
  a.ang = m.d_nbr_ang;
  a.rad_off = m.d_rad_off;
  a.ang_off = m.d_ang_off;
  a.max_rad = m.max_rad;
  a.max_ang = m.max_ang;
  a.n = n;
  a.x = m.d_x;
  size_t lds = sizeof(float) * (64 * (size_t)kPartStride + 5 * (size_t)m.max_ang);
  hipLaunchKernelGGL(k_desc_fwd, dim3(n), dim3(64), lds, st, a, m.dp, m.geo);
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
  size_t lds = sizeof(double) * 3 * (size_t)m.max_rad + sizeof(float) * (size_t)m.stride +
               sizeof(float) * 7 * (size_t)m.max_ang + sizeof(int) * 2 * (size_t)m.max_ang;
  hipLaunchKernelGGL(k_desc_bwd, dim3(n), dim3(64), lds, st, a, m.dp, m.geo);
  return hipGetLastError();
}

hipError_t launch_force_gather(nnp_model& m, int n, double* forces, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_force_gather, dim3((unsigned)((16 * (int64_t)n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     m.d_contrib, m.d_self,
                     m.d_rad_off, m.d_slot_atom, n, m.S, m.max_rad, forces, m.d_link_F);
  return hipGetLastError();
}

}  // namespace nnp
