// Symmetry-function descriptors (forward) and their adjoint (backward with
// the FP64 force scatter), the force gather with the energy reduction, and
// the link-atom chain rule.  The descriptors are those of the ANI family of
// models the paper runs and benchmarks (Methods; performance section); the
// adjoint gives F = -grad E (Theory, eq. 2).
//
// The forward runs one 16-lane row per atom (k_desc_fwd_rows, default), one
// wavefront per atom (k_desc_fwd), or several atoms per wavefront with the
// lanes balanced over chunks of all their work (k_desc_fwd_pool, for many
// elements); the adjoint one wavefront (or half of one) per atom.  An output block is either the radial block of one neighbour
// species (16 outputs) or the angular block of one unordered species pair
// (8 x 4 outputs).
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
#include <climits>

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

__device__ __forceinline__ Geo displacement(const float4& pi, const float4& pj, const MinImage& b) {
  Geo o;
  float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
  if (b.on) {
    dx -= b.L[0] * rintf(dx * b.iL[0]);
    dy -= b.L[1] * rintf(dy * b.iL[1]);
    dz -= b.L[2] * rintf(dz * b.iL[2]);
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
  c.inv2rc = p.inv2rc;
  c.inv2rca = p.inv2rca;
  c.dfc_r = p.dfc_r;
  c.dfc_a = p.dfc_a;
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
  const int* order;        // bin-major visiting order of the slots
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
  const int i = a.order[xcd_block(blockIdx.x, gridDim.x)];
  const int lane = threadIdx.x;
  const Consts c = make_consts(p);
  const float4 pi = a.spos[i];
  const MinImage mi = min_image_at(geo, i);
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
        Geo d = displacement(pi, a.spos[rrow[t]], mi);
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
    Geo d = displacement(pi, a.spos[arow[u]], mi);
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

// ---------------------------------------------------------------------------
// Row kernels: one 16-lane DPP row per atom, four atoms per wavefront.
//
// The lanes of a row split an output block's pairs (radial: strided over the
// species segment; angular: a contiguous range of the class's (j, k) pairs),
// each lane accumulating the whole block in registers; the row then sums the
// block across its 16 lanes with a transposing butterfly (every step halves
// the values a lane holds, so 16 values cost 15 exchanges and 32 cost 30),
// leaving lane l with outputs [l B/16, (l+1) B/16).  The exchanges are DPP
// row permutations: mirror (l <-> 15-l), half-mirror (l <-> 7-l within each
// half) and the quad swaps xor 2 and xor 1; the pairings are disjoint, so
// after four steps every lane's values cover all 16 lanes exactly once.

// Sum N values over the L = 16 or 8 lanes of a row; lane `sub` ends with
// totals [sub N/L, (sub+1) N/L) in v[0 .. N/L).  An 8-lane row is half of a
// DPP row, whose half-mirror pairs lanes across bit 2 within each half.
template <int N, int L>
__device__ __forceinline__ void row_reduce(float* v, int sub) {
  if constexpr (L == 16) {
    halve<N / 2, kDppMirror>(v, sub & 8);
    halve<N / 4, kDppHalfMirror>(v, sub & 4);
    halve<N / 8, kDppXor2>(v, sub & 2);
    halve<N / 16, kDppXor1>(v, sub & 1);
  } else {
    static_assert(L == 8, "row width");
    halve<N / 2, kDppHalfMirror>(v, sub & 4);
    halve<N / 4, kDppXor2>(v, sub & 2);
    halve<N / 8, kDppXor1>(v, sub & 1);
  }
}

// Start of a lane's contiguous range [r0, r1) of T unordered pairs within a
// class, decoded to (j, k): same species: k-major over j < k; different
// species: j-major over (j, k).
__device__ __forceinline__ void pair_start(int r0, bool same, int nB, int* j, int* k) {
  if (same) {
    int kk = (int)((1.f + __builtin_amdgcn_sqrtf(1.f + 8.f * (float)r0)) * 0.5f);
    if (kk * (kk - 1) / 2 > r0) --kk;      // the sqrt is within an ulp: one step each way
    if ((kk + 1) * kk / 2 <= r0) ++kk;
    *k = kk;
    *j = r0 - kk * (kk - 1) / 2;
  } else {
    const int jj = (int)(((float)r0 + 0.5f) * __builtin_amdgcn_rcpf((float)max(nB, 1)));
    *j = jj;
    *k = r0 - jj * nB;
  }
}

// L lanes per atom (16 or 8), 256 / L atoms per 256-thread workgroup.
template <int L>
__global__ __launch_bounds__(256) void k_desc_fwd_rows(FwdArgs a, DescParams p, Geometry geo) {
  constexpr int kAtoms = 256 / L;
  extern __shared__ float4 smem_r[];
  const int row = threadIdx.x / L, sub = threadIdx.x % L;
  float4* G = smem_r + row * a.max_ang;                                      // (u, r hq)
  float* W = reinterpret_cast<float*>(smem_r + kAtoms * a.max_ang) + row * a.max_ang;  // fc sq_pref
  const int li = xcd_block(blockIdx.x, gridDim.x) * kAtoms + row;   // place in the visiting order
  const bool valid = li < a.n;
  const Consts c = make_consts(p);
  const int S1 = p.S + 1;
  const int ii = valid ? a.order[li] : 0;
  const float4 pi = a.spos[ii];
  const MinImage mi = min_image_at(geo, ii);
  const int* roff = a.rad_off + (int64_t)ii * S1;
  const int* aoff = a.ang_off + (int64_t)ii * S1;
  const int* rrow = a.rad + (int64_t)ii * a.max_rad;
  const int* arow = a.ang + (int64_t)ii * a.max_ang;
  float* xo = a.x + (int64_t)ii * p.stride;

  // angular neighbour geometry of this row's atom
  const int na = valid ? aoff[p.S] : 0;
  for (int u = sub; u < na; u += L) {
    Geo d = displacement(pi, a.spos[arow[u]], mi);
    G[u] = make_float4(d.dx * d.ir, d.dy * d.ir, d.dz * d.ir, d.r * p.hq_eta_a);
    W[u] = (0.5f * cos_rev(d.r * c.inv2rca) + 0.5f) * p.sq_pref;
  }

  // radial blocks
  for (int s = 0; s < p.S; ++s) {
    float acc[kRadShifts];
#pragma unroll
    for (int k = 0; k < kRadShifts; ++k) acc[k] = 0.f;
    const int t1 = valid ? roff[s + 1] : 0;
    for (int t = (valid ? roff[s] : 0) + sub; t < t1; t += L) {
#pragma clang fp contract(off)   // keep r sq in a register: one SGPR operand per shift
      Geo d = displacement(pi, a.spos[rrow[t]], mi);
      const float fc = fmaf(0.5f, cos_rev(d.r * c.inv2rc), 0.5f);
      const float rs = d.r * p.sq_eta_r;
#pragma unroll
      for (int k = 0; k < kRadShifts; ++k) {
        const float tt = rs - p.rad_shift_s[k];
        acc[k] = fmaf(ex2(-(tt * tt)), fc, acc[k]);
      }
    }
    row_reduce<kRadShifts, L>(acc, sub);
    if (valid) {
      if constexpr (L == 16) xo[s * kRadShifts + sub] = acc[0];
      else *reinterpret_cast<float2*>(xo + s * kRadShifts + 2 * sub) = make_float2(acc[0], acc[1]);
    }
  }
  __syncthreads();

  // angular blocks
  for (int q = 0; q < p.P; ++q) {
    const int sa = p.pair_a[q], sb = p.pair_b[q];
    const bool same = sa == sb;
    int oa = 0, ob = 0, nA = 0, nB = 0;
    if (valid) {
      oa = aoff[sa];
      nA = aoff[sa + 1] - oa;
      ob = aoff[sb];
      nB = aoff[sb + 1] - ob;
    }
    const int T = same ? nA * (nA - 1) / 2 : nA * nB;
    const int r0 = (T * sub) / L, r1 = (T * (sub + 1)) / L;
    float acc[kAngShifts * kAngSects];
#pragma unroll
    for (int e = 0; e < kAngShifts * kAngSects; ++e) acc[e] = 0.f;
    if (r0 < r1) {
      int j, k;
      pair_start(r0, same, nB, &j, &k);
      const int kbase = same ? oa : ob;
      for (int r = r0; r < r1; ++r) {
        const float4 gj = G[oa + j], gk = G[kbase + k];
        const float F = W[oa + j] * W[kbase + k];
        const float cs = gj.x * gk.x + gj.y * gk.y + gj.z * gk.z;
        const float ct = 0.95f * cs;
        const float sn = __builtin_amdgcn_sqrtf(1.f - ct * ct);
        const float rb = gj.w + gk.w;
        float A[kAngSects];
#pragma unroll
        for (int n = 0; n < kAngSects; ++n) {
          const float base = 1.f + ct * p.cos_sect[n] + sn * p.sin_sect[n];
          A[n] = F * ex2(p.zeta * lg2(base));
        }
#pragma unroll
        for (int m = 0; m < kAngShifts; ++m) {
          const float tt = rb - p.ang_shift_s[m];
          const float B = ex2(-(tt * tt));
#pragma unroll
          for (int n = 0; n < kAngSects; ++n) acc[m * kAngSects + n] = fmaf(B, A[n], acc[m * kAngSects + n]);
        }
        if (same) {
          if (++j == k) { j = 0; ++k; }
        } else {
          if (++k == nB) { k = 0; ++j; }
        }
      }
    }
    row_reduce<kAngShifts * kAngSects, L>(acc, sub);
    if (valid) {
      float* dst = xo + p.S * kRadShifts + q * kAngShifts * kAngSects;
      if constexpr (L == 16)
        *reinterpret_cast<float2*>(dst + 2 * sub) = make_float2(acc[0], acc[1]);
      else
        *reinterpret_cast<float4*>(dst + 4 * sub) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
  }
}

// ---------------------------------------------------------------------------
// Pool kernel: AW atoms per wavefront, the lanes balanced over the work of
// all of them.
//
// The radial neighbours of one (atom, neighbour species) and the angular
// pairs of one (atom, species-pair class) form a unit.  The wavefront cuts
// its units into chunks of at most C items, C being (within a few steps) the
// smallest size for which the chunks fit its 64 lanes, and each lane sums one
// chunk's block in registers.  The chunks of a unit then add up pairwise in
// a tree (chunk c + d into chunk c for c a multiple of 2d, d = 1, 2, 4, ...,
// 16 values at a time through LDS), and the unit's first chunk stores the
// block in the descriptor row.
//
// With several elements a class holds few pairs (about 14 per class for
// H/C/N/O molecules against 17 angular neighbours): the row kernels then
// leave most lanes of a row idle and pay a 32-value cross-lane reduction per
// class, which this kernel avoids.  Adding the partials with LDS float
// atomics instead was several times slower.  The radial phase runs first,
// with the first pass of the angular geometry already loaded into registers,
// so that the partial rows can share LDS with the angular geometry (each is
// dead while the other is live).
constexpr int kPoolPitch = 20;   // LDS row of one lane's 16 partial sums (16-byte aligned)

// Inclusive prefix sum / maximum over the 64 lanes with DPP: row shifts
// within each 16-lane row, then the row broadcasts of lanes 15 and 31.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <bool MAX>
__device__ __forceinline__ int wave_scan_dpp(int v) {
  // out-of-row sources read as the identity (0 for the sums; counts and
  // packed owners here are never negative, so 0 also serves the maximum)
#define NNP_SCAN_STEP(CTRL, RM)                                               \
  {                                                                           \
    const int t = __builtin_amdgcn_update_dpp(0, v, CTRL, RM, 0xF, true);     \
    v = MAX ? max(v, t) : v + t;                                              \
  }
  NNP_SCAN_STEP(kDppRowShr1, 0xF)
  NNP_SCAN_STEP(kDppRowShr2, 0xF)
  NNP_SCAN_STEP(kDppRowShr4, 0xF)
  NNP_SCAN_STEP(kDppRowShr8, 0xF)
  NNP_SCAN_STEP(kDppRowBcast15, 0xA)
  NNP_SCAN_STEP(kDppRowBcast31, 0xC)
#undef NNP_SCAN_STEP
  return v;
}

__device__ __forceinline__ int wave_total(int v) {
  return __builtin_amdgcn_readlane(wave_scan_dpp<false>(v), 63);
}

// ceil(x / C) for 0 <= x < 2^20 and C >= 1, with rC = 1 / C: the FP32
// quotient is within one of the true one, and one correction each way fixes it.
__device__ __forceinline__ int ceil_div(int x, int C, float rC) {
  if (x <= 0) return 0;
  const int y = x - 1;
  int q = (int)((float)y * rC);
  q -= q * C > y ? 1 : 0;
  q += (q + 1) * C <= y ? 1 : 0;
  return q + 1;
}

// Chunk size for unit sizes cnt (one unit per lane, 0 elsewhere): with U
// non-empty units and N items, C = ceil(N / (64 - U)) always fits, since the
// chunk count is below N / C + U; smaller sizes are tried while they still fit.
__device__ __forceinline__ int pool_chunk(int cnt) {
  const int N = wave_total(cnt);
  if (N == 0) return 0;
  const int U = (int)__popcll(__ballot(cnt > 0));
  int C = (N + 63 - U) / (64 - U);   // uniform: scalar arithmetic
  for (int step = 0; step < 3 && C > 1; ++step) {
    const int k = ceil_div(cnt, C - 1, __builtin_amdgcn_rcpf((float)(C - 1)));
    if (wave_total(k) > 64) break;
    --C;
  }
  return C;
}

// The wavefronts of a pool workgroup work independently, each in its own LDS
// slice, and synchronise only among their own lanes: LDS accesses of one
// wavefront complete in order, so keeping the compiler from moving them
// across this point is enough.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Hands the chunks out to the lanes in unit order: lane l < K gets unit *unit
// (the lane that holds it), chunk *chunk of that unit and the unit's chunk
// count *nunit; other lanes get unit -1.  Returns the largest chunk count.
__device__ __forceinline__ int pool_assign(int cnt, int C, int lane, int* owner, int* unit, int* chunk,
                                           int* nunit) {
  const int nch = C > 0 ? ceil_div(cnt, C, __builtin_amdgcn_rcpf((float)C)) : 0;
  const int incl = wave_scan_dpp<false>(nch);
  const int K = __builtin_amdgcn_readlane(incl, 63);
  const int excl = incl - nch;
  owner[lane] = 0;
  wave_sync();
  if (nch > 0) owner[excl] = ((lane + 1) << 8) | excl;
  wave_sync();
  const int o = wave_scan_dpp<true>(owner[lane]);
  *unit = lane < K ? (o >> 8) - 1 : -1;
  *chunk = lane < K ? lane - (o & 255) : 0;
  *nunit = __shfl(nch, max(*unit, 0), 64);
  return __builtin_amdgcn_readlane(wave_scan_dpp<true>(nch), 63);
}

// Pairwise tree over the chunks of each unit (chunks of a unit sit on
// consecutive lanes): chunk c + d adds into chunk c for c a multiple of 2d,
// through this lane's LDS row, until chunk 0 holds the unit's sums.
__device__ __forceinline__ void pool_tree16(float* v, float* part, int lane, int unit, int chunk, int nunit,
                                            int maxn) {
  for (int d = 1; d < maxn; d *= 2) {
    wave_sync();
    if (unit >= 0 && (chunk & (2 * d - 1)) == d) {
      float4* row = reinterpret_cast<float4*>(part + lane * kPoolPitch);
#pragma unroll
      for (int e = 0; e < 4; ++e) row[e] = make_float4(v[4 * e], v[4 * e + 1], v[4 * e + 2], v[4 * e + 3]);
    }
    wave_sync();
    if (unit >= 0 && (chunk & (2 * d - 1)) == 0 && chunk + d < nunit) {
      const float4* row = reinterpret_cast<const float4*>(part + (lane + d) * kPoolPitch);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float4 w = row[e];
        v[4 * e] += w.x;
        v[4 * e + 1] += w.y;
        v[4 * e + 2] += w.z;
        v[4 * e + 3] += w.w;
      }
    }
  }
}

__device__ __forceinline__ void store16(float* dst, const float* v) {
  float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
  for (int e = 0; e < 4; ++e) d4[e] = make_float4(v[4 * e], v[4 * e + 1], v[4 * e + 2], v[4 * e + 3]);
}

template <int AW>
__global__ __launch_bounds__(256) void k_desc_fwd_pool(FwdArgs a, DescParams p, Geometry geo) {
  static_assert(AW >= 1 && AW * kMaxPairs <= 40, "units must leave lanes for the chunks");
  extern __shared__ float4 smem_pool[];
  const int S = p.S, P = p.P, S1 = S + 1;
  // per wavefront: [angular geometry | partial rows (aliased: never live together)] [owner]
  const int area = (max(AW * a.max_ang * 5, 64 * kPoolPitch) + 3) & ~3;   // floats
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  float4* smem_p = smem_pool + wave * ((area + 64) / 4);
  float4* G = smem_p;                                             // [AW][max_ang] (u, r hq)
  float* W = reinterpret_cast<float*>(G + AW * a.max_ang);        // [AW][max_ang] fc sq_pref
  float* part = reinterpret_cast<float*>(smem_p);                 // [64][kPoolPitch]
  int* owner = reinterpret_cast<int*>(smem_p) + area;             // [64]
  const int li0 = (xcd_block(blockIdx.x, gridDim.x) * 4 + wave) * AW;
  const Consts c = make_consts(p);
  int slot[AW], na[AW];
  int nat = 0;
#pragma unroll
  for (int t = 0; t < AW; ++t) {
    slot[t] = li0 + t < a.n ? a.order[li0 + t] : 0;
    na[t] = li0 + t < a.n ? a.ang_off[(int64_t)slot[t] * S1 + S] : 0;
    nat += na[t];
  }
  auto atom_of = [&](int t) {
    int ii = slot[0];
#pragma unroll
    for (int k = 1; k < AW; ++k) ii = t == k ? slot[k] : ii;
    return ii;
  };

  // ---- angular units (lane t * kMaxPairs + q), set up first so that their
  // loads and the first pass of the geometry loads overlap the radial phase
  uint64_t pairs = 0;   // species pairs of the classes, four bits each (uniform)
#pragma unroll
  for (int k = 0; k < kMaxPairs; ++k) pairs |= (uint64_t)(p.pair_a[k] | (p.pair_b[k] << 2)) << (4 * k);
  int T = 0, oa = 0, kb = 0, nB = 0, same = 0;
  {
    const int t = lane / kMaxPairs, q = lane % kMaxPairs;
    if (t < AW && q < P && li0 + t < a.n) {
      const int code = (int)(pairs >> (4 * q)) & 15;
      const int sa = code & 3, sb = code >> 2;
      const int ii = atom_of(t);
      const int* aoff = a.ang_off + (int64_t)ii * S1;
      oa = aoff[sa];
      const int nA = aoff[sa + 1] - oa;
      const int ob = aoff[sb];
      nB = aoff[sb + 1] - ob;
      same = sa == sb;
      kb = same ? oa : ob;
      T = same ? nA * (nA - 1) / 2 : nA * nB;
      if (T == 0) {   // no pairs in this class
        const float zero[kRadShifts] = {};
        float* dst = a.x + (int64_t)ii * p.stride + S * kRadShifts + q * kAngShifts * kAngSects;
        store16(dst, zero);
        store16(dst + 16, zero);
      }
    }
  }
  // angular neighbour geometry, flattened over the atoms: the first pass is
  // loaded now and stored to LDS after the radial phase (whose partial rows
  // share that LDS)
  auto split = [&](int f, int* tt, int* uu) {
    int t = 0, u = f;
#pragma unroll
    for (int k = 0; k + 1 < AW; ++k)
      if (t == k && u >= na[k]) { u -= na[k]; t = k + 1; }
    *tt = t;
    *uu = u;
  };
  int g_t = 0, g_u = 0, g_ii = 0;
  float4 g_pi = make_float4(0.f, 0.f, 0.f, 0.f), g_pj = g_pi;
  if (lane < nat) {
    split(lane, &g_t, &g_u);
    g_ii = atom_of(g_t);
    g_pi = a.spos[g_ii];
    g_pj = a.spos[a.ang[(int64_t)g_ii * a.max_ang + g_u]];
  }

  // ---- radial units (lane t * kMaxSpecies + s) and chunks
  {
    const int t = lane / kMaxSpecies, s = lane % kMaxSpecies;
    int beg = 0, cnt = 0, ii = 0;
    if (t < AW && s < S && li0 + t < a.n) {
      ii = atom_of(t);
      const int* roff = a.rad_off + (int64_t)ii * S1;
      beg = roff[s];
      cnt = roff[s + 1] - beg;
      if (cnt == 0) {   // no neighbours of this species
        const float zero[kRadShifts] = {};
        store16(a.x + (int64_t)ii * p.stride + s * kRadShifts, zero);
      }
    }
    const int C = pool_chunk(cnt);
    int unit, chunk, nunit;
    const int maxn = pool_assign(cnt, C, lane, owner, &unit, &chunk, &nunit);
    const int src = max(unit, 0);
    const int ub = __shfl(beg, src, 64), ue = __shfl(beg + cnt, src, 64), ui = __shfl(ii, src, 64);
    float acc[kRadShifts];
#pragma unroll
    for (int k = 0; k < kRadShifts; ++k) acc[k] = 0.f;
    if (unit >= 0) {
      const int b0 = ub + chunk * C, b1 = min(b0 + C, ue);
      const float4 pi = a.spos[ui];
      const MinImage mi = min_image_at(geo, ui);
      const int* rrow = a.rad + (int64_t)ui * a.max_rad;
      for (int q = b0; q < b1; ++q) {
#pragma clang fp contract(off)   // keep r sq in a register: one SGPR operand per shift
        const Geo d = displacement(pi, a.spos[rrow[q]], mi);
        const float fc = fmaf(0.5f, cos_rev(d.r * c.inv2rc), 0.5f);
        const float rs = d.r * p.sq_eta_r;
#pragma unroll
        for (int k = 0; k < kRadShifts; ++k) {
          const float tt = rs - p.rad_shift_s[k];
          acc[k] = fmaf(ex2(-(tt * tt)), fc, acc[k]);
        }
      }
    }
    pool_tree16(acc, part, lane, unit, chunk, nunit, maxn);
    if (unit >= 0 && chunk == 0) store16(a.x + (int64_t)ui * p.stride + (src % kMaxSpecies) * kRadShifts, acc);
  }
  wave_sync();

  // ---- angular geometry to LDS
  for (int f = lane; f < nat; f += 64) {
    if (f >= 64) {
      split(f, &g_t, &g_u);
      g_ii = atom_of(g_t);
      g_pi = a.spos[g_ii];
      g_pj = a.spos[a.ang[(int64_t)g_ii * a.max_ang + g_u]];
    }
    const Geo d = displacement(g_pi, g_pj, min_image_at(geo, g_ii));
    G[g_t * a.max_ang + g_u] = make_float4(d.dx * d.ir, d.dy * d.ir, d.dz * d.ir, d.r * p.hq_eta_a);
    W[g_t * a.max_ang + g_u] = (0.5f * cos_rev(d.r * c.inv2rca) + 0.5f) * p.sq_pref;
  }
  wave_sync();

  // ---- angular chunks
  const int C = pool_chunk(T);
  int unit, chunk, nunit;
  const int maxn = pool_assign(T, C, lane, owner, &unit, &chunk, &nunit);
  const int src = max(unit, 0);
  const int uT = __shfl(T, src, 64), uoa = __shfl(oa, src, 64), ukb = __shfl(kb, src, 64);
  const int unB = __shfl(nB, src, 64), usame = __shfl(same, src, 64);
  const int ut = src / kMaxPairs;
  float acc[kAngShifts * kAngSects];
#pragma unroll
  for (int e = 0; e < kAngShifts * kAngSects; ++e) acc[e] = 0.f;
  if (unit >= 0) {
    const float4* Gt = G + ut * a.max_ang;
    const float* Wt = W + ut * a.max_ang;
    const int r0 = chunk * C, r1 = min(r0 + C, uT);
    // (inner, outer) walk: same species k-major over j < k (inner j, limit k),
    // two species j-major (inner k, limit nB)
    int j, k;
    pair_start(r0, usame != 0, unB, &j, &k);
    int in = usame ? j : k, out = usame ? k : j;
    for (int r = r0; r < r1; ++r) {
      const int jj = usame ? in : out, kk = usame ? out : in;
      const float4 gj = Gt[uoa + jj], gk = Gt[ukb + kk];
      const float F = Wt[uoa + jj] * Wt[ukb + kk];
      const float cs = gj.x * gk.x + gj.y * gk.y + gj.z * gk.z;
      const float ct = 0.95f * cs;
      const float sn = __builtin_amdgcn_sqrtf(1.f - ct * ct);
      const float rb = gj.w + gk.w;
      float A[kAngSects];
#pragma unroll
      for (int n = 0; n < kAngSects; ++n) {
        const float base = 1.f + ct * p.cos_sect[n] + sn * p.sin_sect[n];
        A[n] = F * ex2(p.zeta * lg2(base));
      }
#pragma unroll
      for (int m = 0; m < kAngShifts; ++m) {
        const float tt = rb - p.ang_shift_s[m];
        const float B = ex2(-(tt * tt));
#pragma unroll
        for (int n = 0; n < kAngSects; ++n) acc[m * kAngSects + n] = fmaf(B, A[n], acc[m * kAngSects + n]);
      }
      ++in;
      const bool wrap = in == (usame ? out : unB);
      in = wrap ? 0 : in;
      out += wrap ? 1 : 0;
    }
  }
  // the unit sums in two halves of 16 (the geometry is dead from here on)
  constexpr int B = kAngShifts * kAngSects, H = B / 2;
  float* dst = a.x + (int64_t)atom_of(ut) * p.stride + S * kRadShifts + (src % kMaxPairs) * B;
  pool_tree16(acc, part, lane, unit, chunk, nunit, maxn);
  if (unit >= 0 && chunk == 0) store16(dst, acc);
  pool_tree16(acc + H, part, lane, unit, chunk, nunit, maxn);
  if (unit >= 0 && chunk == 0) store16(dst + H, acc + H);
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
  const int* order;        // bin-major visiting order of the slots
  const float4* spos;
  const int* rad;
  const int* ang;
  const int* angpos;
  const int* rad_off;
  const int* ang_off;
  int max_rad, max_ang, n;
  const float* g;
  float3* contrib;   // [n][max_rad]
  double* self;      // [n][3]
};

// Sum over the LANES lanes of one atom (xor offsets below LANES stay inside it).
template <int LANES>
__device__ __forceinline__ double part_sum_d(double v) {
#pragma unroll
  for (int off = LANES / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Bytes of LDS per atom of the adjoint: FP64 slots, the dE/dx row, padding to
// 16 bytes, two float4 records per angular neighbour (a multiple of 16).
__host__ __device__ __forceinline__ size_t bwd_lds_per_atom(int max_rad, int max_ang, int stride) {
  return sizeof(double) * 3 * (size_t)max_rad + sizeof(float) * (size_t)stride +
         sizeof(float) * 2 * ((size_t)max_rad & 1) + sizeof(float4) * 2 * (size_t)max_ang;
}

// LANES lanes per atom: 64 (one atom per wavefront) or 32 (two atoms per
// wavefront, so that the ~153 triplets of an atom in water fill the lanes
// with less rounding).  WIDE: the centre's place in each neighbour's list is
// counted with wide loads instead of a binary search (step 5).
template <int LANES, bool WIDE>
__global__ __launch_bounds__(64) void k_desc_bwd(BwdArgs a, DescParams p, Geometry geo) {
  constexpr int APW = 64 / LANES;   // atoms per wavefront
  extern __shared__ double smem_d[];
  const int part = threadIdx.x / LANES;
  const int lane = threadIdx.x % LANES;
  char* region = reinterpret_cast<char*>(smem_d) + part * bwd_lds_per_atom(a.max_rad, a.max_ang, p.stride);
  double* sx = reinterpret_cast<double*>(region);   // per radial neighbour, FP64
  double* sy = sx + a.max_rad;
  double* sz = sy + a.max_rad;
  float* gl = reinterpret_cast<float*>(sz + a.max_rad);   // [stride] dE/dx of the centre
  // angular neighbours: (u, r hq) and (fc sq_pref, dfc sq_pref, 1/r, radial position * 8 + species)
  float4* G1 = reinterpret_cast<float4*>(gl + p.stride + 2 * (a.max_rad & 1));   // 16-byte aligned
  float4* G2 = G1 + a.max_ang;
  const int li = xcd_block(blockIdx.x, gridDim.x) * APW + part;
  const bool valid = li < a.n;
  const int i = valid ? a.order[li] : 0;
  const Consts c = make_consts(p);
  const float4 pi = a.spos[i];
  const MinImage mi = min_image_at(geo, i);
  const int S1 = p.S + 1;
  const int nr = valid ? a.rad_off[(int64_t)i * S1 + p.S] : 0;
  const int na = valid ? a.ang_off[(int64_t)i * S1 + p.S] : 0;
  const int* rrow = a.rad + (int64_t)i * a.max_rad;
  const int* arow = a.ang + (int64_t)i * a.max_ang;
  float fx = 0.f, fy = 0.f, fz = 0.f;   // this lane's share of the centre's total

  // 1. dE/dx row
  if (valid) {
    const float4* g4 = reinterpret_cast<const float4*>(a.g + (int64_t)i * p.stride);
    float4* l4 = reinterpret_cast<float4*>(gl);
    for (int q = lane; q < p.D / 4; q += LANES) l4[q] = g4[q];
  }
  // 3. angular neighbour geometry (before the barrier, together with 1.)
  for (int u = lane; u < na; u += LANES) {
    const float4 pj = a.spos[arow[u]];
    Geo d = displacement(pi, pj, mi);
    const float arg = d.r * c.inv2rca;
    G1[u] = make_float4(d.dx * d.ir, d.dy * d.ir, d.dz * d.ir, d.r * p.hq_eta_a);
    G2[u] = make_float4(fmaf(0.5f, cos_rev(arg), 0.5f) * p.sq_pref, c.dfc_a * sin_rev(arg) * p.sq_pref, d.ir,
                        __int_as_float(a.angpos[(int64_t)i * a.max_ang + u] * 8 + __float_as_int(pj.w)));
  }
  __syncthreads();
  // 2. radial pairs
  {
    const float c1 = p.c1_rad;   // d/dr of -(r sq - Rs sq)^2 per (r sq - Rs sq), in ln units
    for (int t = lane; t < nr; t += LANES) {
#pragma clang fp contract(off)   // keep r sq in a register: one SGPR operand per shift
      const float4 pj = a.spos[rrow[t]];
      const int sj = __float_as_int(pj.w);
      Geo d = displacement(pi, pj, mi);
      const float arg = d.r * c.inv2rc;
      const float fc = fmaf(0.5f, cos_rev(arg), 0.5f);
      const float dfc = c.dfc_r * sin_rev(arg);
      const float rs = d.r * p.sq_eta_r;
      const float4* g4 = reinterpret_cast<const float4*>(gl + sj * kRadShifts);
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int q = 0; q < kRadShifts / 4; ++q) {
        const float4 gv = g4[q];
        const float gk[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float tt = rs - p.rad_shift_s[4 * q + u];
          const float B = gk[u] * ex2(-(tt * tt));
          s0 += B;
          s1 = fmaf(B, tt, s1);
        }
      }
      const float dTdr = fmaf(dfc, s0, c1 * fc * s1);
      const float w = dTdr * d.ir;
      const float vx = w * d.dx, vy = w * d.dy, vz = w * d.dz;
      sx[t] = vx;
      sy[t] = vy;
      sz[t] = vz;
      fx += vx; fy += vy; fz += vz;
    }
  }
  __syncthreads();
  // 4. angular triplets (j < k, k-major), a contiguous range per lane
  const int T = na * (na - 1) / 2;
  const int r0 = (int)(((int64_t)T * lane) / LANES);
  const int r1 = (int)(((int64_t)T * (lane + 1)) / LANES);
  if (r0 < r1) {
#pragma clang fp contract(off)
    int k = (int)((1.f + __builtin_amdgcn_sqrtf(1.f + 8.f * (float)r0)) * 0.5f);
    if (k * (k - 1) / 2 > r0) --k;
    if ((k + 1) * k / 2 <= r0) ++k;
    int j = r0 - k * (k - 1) / 2;
    const float c_sdr = p.c_sdr;     // d rbar-term per (rbar sa - Ra sa), sa = 2 hq
    const float c_dc = p.zeta * 0.95f;
    float kx = 0.f, ky = 0.f, kz = 0.f;   // running total of the current k
    float4 k1 = G1[k], k2 = G2[k];
    for (int r = r0; r < r1; ++r) {
      const float4 j1 = G1[j], j2 = G2[j];
      const int wj = __float_as_int(j2.w), wk = __float_as_int(k2.w);
      const int sj = wj & 7, sk = wk & 7;                   // sj <= sk (rows are grouped by species)
      const int q = (int)(p.class_tab >> (4 * (4 * sj + sk))) & 15;
      const float4* g4 = reinterpret_cast<const float4*>(gl + p.S * kRadShifts + q * kAngShifts * kAngSects);
      const float cs = fmaf(j1.x, k1.x, fmaf(j1.y, k1.y, j1.z * k1.z));
      const float ct = 0.95f * cs;
      const float s2 = fmaf(-ct, ct, 1.f);
      const float ist = rsq(s2);
      const float st = s2 * ist;
      const float qq = ct * ist;
      const float rb = j1.w + k1.w;
      float A[kAngSects], Ab[kAngSects];
#pragma unroll
      for (int n = 0; n < kAngSects; ++n) {
        const float base = fmaf(st, p.sin_sect[n], fmaf(ct, p.cos_sect[n], 1.f));
        const float An = ex2(p.zeta * lg2(base));
        A[n] = An;
        Ab[n] = An * __builtin_amdgcn_rcpf(base);
      }
      float h[kAngSects] = {0.f, 0.f, 0.f, 0.f};
      float sdr = 0.f;
#pragma unroll
      for (int m = 0; m < kAngShifts; ++m) {
        const float4 gv = g4[m];
        const float tt = rb - p.ang_shift_s[m];
        const float B = ex2(-(tt * tt));
        h[0] = fmaf(gv.x, B, h[0]);
        h[1] = fmaf(gv.y, B, h[1]);
        h[2] = fmaf(gv.z, B, h[2]);
        h[3] = fmaf(gv.w, B, h[3]);
        const float km = fmaf(gv.x, A[0], fmaf(gv.y, A[1], fmaf(gv.z, A[2], gv.w * A[3])));
        sdr = fmaf(tt * B, km, sdr);
      }
      float SA = 0.f, SP = 0.f, SQ = 0.f;
#pragma unroll
      for (int n = 0; n < kAngSects; ++n) {
        SA = fmaf(h[n], A[n], SA);
        const float wn = h[n] * Ab[n];
        SP = fmaf(wn, p.cos_sect[n], SP);
        SQ = fmaf(wn, p.sin_sect[n], SQ);
      }
      const float F = j2.x * k2.x;
      const float dTdc = F * c_dc * fmaf(-qq, SQ, SP);
      const float hdr = 0.5f * F * c_sdr * sdr;
      const float dTdrj = fmaf(j2.y * k2.x, SA, hdr);
      const float dTdrk = fmaf(j2.x * k2.y, SA, hdr);
      const float cj = dTdc * j2.z, ck = dTdc * k2.z;
      const float vjx = fmaf(cj, fmaf(-cs, j1.x, k1.x), dTdrj * j1.x);
      const float vjy = fmaf(cj, fmaf(-cs, j1.y, k1.y), dTdrj * j1.y);
      const float vjz = fmaf(cj, fmaf(-cs, j1.z, k1.z), dTdrj * j1.z);
      const float vkx = fmaf(ck, fmaf(-cs, k1.x, j1.x), dTdrk * k1.x);
      const float vky = fmaf(ck, fmaf(-cs, k1.y, j1.y), dTdrk * k1.y);
      const float vkz = fmaf(ck, fmaf(-cs, k1.z, j1.z), dTdrk * k1.z);
      const int pj = wj >> 3;
      unsafeAtomicAdd(sx + pj, (double)vjx);
      unsafeAtomicAdd(sy + pj, (double)vjy);
      unsafeAtomicAdd(sz + pj, (double)vjz);
      kx += vkx; ky += vky; kz += vkz;
      fx += vjx + vkx;
      fy += vjy + vky;
      fz += vjz + vkz;
      if (++j == k || r + 1 == r1) {   // k changes (or the range ends): flush its total
        const int pk = wk >> 3;
        unsafeAtomicAdd(sx + pk, (double)kx);
        unsafeAtomicAdd(sy + pk, (double)ky);
        unsafeAtomicAdd(sz + pk, (double)kz);
        kx = ky = kz = 0.f;
        if (j == k) {
          j = 0;
          ++k;
          if (r + 1 < r1) {
            k1 = G1[k];
            k2 = G2[k];
          }
        }
      }
    }
  }
  __syncthreads();
  // 5. each neighbour's total goes to the centre's slot in the neighbour's list:
  // in j's species segment [lo, hi) (sorted by slot) the centre sits after the
  // entries below i.  A binary search finds it with one dependent load per
  // halving.  The WIDE form counts the entries below i 32 at a time from
  // eight independent aligned 16-byte loads: one or two round trips instead
  // of about six, for four times the bytes.  That wins when the lists are
  // far beyond the caches (261k atoms: 687 -> 642 us) and loses while they
  // are cache-resident (12k atoms: 34 -> 42 us), so it is a tuned variant.
  const int si = __float_as_int(pi.w);
  const bool wide = WIDE && (a.max_rad & 3) == 0;   // rows start on 16-byte boundaries
  for (int t = lane; t < nr; t += LANES) {
    const int j = rrow[t];
    const int* jrow = a.rad + (int64_t)j * a.max_rad;
    const int lo = a.rad_off[(int64_t)j * S1 + si], hi = a.rad_off[(int64_t)j * S1 + si + 1];
    int pos = -1;
    if (wide) {
      // lower bound of i in j's segment [lo, hi), 32 entries per round.  The
      // key of entry e is -inf before lo, +inf from hi on and the (sorted)
      // entry in between; keys are monotone, so the groups of four whose
      // first key is below i form a prefix, and the boundary lies in the
      // last of them (or at the next group's first entry).
      for (int e0 = lo & ~3; e0 < hi; e0 += 32) {
        int4 q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)   // a load starting before hi stays inside the row (max_rad % 4 == 0)
          q[u] = e0 + 4 * u < hi ? reinterpret_cast<const int4*>(jrow + e0)[u]
                                 : make_int4(INT_MAX, INT_MAX, INT_MAX, INT_MAX);
        int g = (e0 < lo || q[0].x < i) ? 1 : 0;   // e0 >= lo - 3: only group 0 can start before lo
#pragma unroll
        for (int u = 1; u < 8; ++u) g += q[u].x < i ? 1 : 0;
        int x = 0, at = q[0].x;   // x: keys below i in this round; at: the entry at x
        if (g > 0) {
          const int gs = g - 1;
          int4 sel[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) sel[u] = q[u];
#pragma unroll
          for (int b = 1; b < 8; b <<= 1)   // multiplexer tree: sel[0] = q[gs]
#pragma unroll
            for (int u = 0; u + b < 8; u += 2 * b)
              if (gs & b) sel[u] = sel[u + b];
          int nxt = INT_MAX;   // first entry of group gs + 1
#pragma unroll
          for (int u = 1; u < 8; ++u) nxt = gs + 1 == u ? q[u].x : nxt;
          const int eb = e0 + 4 * gs;
          const int w[4] = {sel[0].x, sel[0].y, sel[0].z, sel[0].w};
          x = 4 * gs + 1;
          at = nxt;
#pragma unroll
          for (int c = 3; c >= 1; --c) {   // keys are monotone: count those below i
            const int e = eb + c;
            const bool less = e < lo || (e < hi && w[c] < i);
            x += less ? 1 : 0;
          }
          at = x == 4 * gs + 1 ? w[1] : x == 4 * gs + 2 ? w[2] : x == 4 * gs + 3 ? w[3] : nxt;
        }
        if (x < 32) {   // the first key >= i is in this round
          if (e0 + x < hi && at == i) pos = e0 + x;
          break;
        }
      }
    } else {
      int l = lo, h = hi - 1;
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (jrow[mid] < i) l = mid + 1; else h = mid;
      }
      if (l <= h && jrow[l] == i) pos = l;
    }
    if (pos >= 0)
      a.contrib[(int64_t)j * a.max_rad + pos] = make_float3((float)-sx[t], (float)-sy[t], (float)-sz[t]);
  }
  // 6. the centre's own total
  double dx = part_sum_d<LANES>((double)fx), dy = part_sum_d<LANES>((double)fy), dz = part_sum_d<LANES>((double)fz);
  if (lane == 0 && valid) {
    a.self[3 * (int64_t)i + 0] = dx;
    a.self[3 * (int64_t)i + 1] = dy;
    a.self[3 * (int64_t)i + 2] = dz;
  }
}

// FP64 energy reduction blocks, appended to the gather's grid (one launch for
// both): with per-tile partials from the network kernel (a single system)
// one block sums them; otherwise block `sys` sums that system's atomic
// energies over its species buckets.  Fixed order, hence deterministic.
struct EnergyArgs {
  const double* part;      // per-tile partials, or null
  const float* e;          // atomic energies in sorted order
  const int* bin_start;    // species buckets [s * n_bins, (s + 1) * n_bins)
  int n_bins, S, tile_rows;
  int mixed;               // the network's narrow species used 16-atom tiles
  int empty;               // no atoms: the energies are zero (the buckets are not read)
  double* out;
  int accumulate;
  int* status;
};

__device__ __forceinline__ void energy_block(const EnergyArgs& ea, int sys) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  if (ea.empty) {
  } else if (ea.part != nullptr) {
    const int narrow = ea.mixed ? narrow_species(ea.bin_start, ea.S, ea.n_bins) : -1;
    int tiles = 0;
    for (int s = 0; s < ea.S; ++s) {
      const int rows = s == narrow ? 16 : ea.tile_rows;
      tiles += (ea.bin_start[(s + 1) * ea.n_bins] - ea.bin_start[s * ea.n_bins] + rows - 1) / rows;
    }
    // eight loads in flight per thread, added in the same order as one at a time
    for (int t0 = threadIdx.x; t0 < tiles; t0 += 8 * kBlock) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = t0 + u * kBlock < tiles ? ea.part[t0 + u * kBlock] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (t0 + u * kBlock < tiles) acc += v[u];
    }
  } else {
    for (int s = 0; s < ea.S; ++s) {
      const int b0 = ea.bin_start[s * ea.n_bins + sys], b1 = ea.bin_start[s * ea.n_bins + sys + 1];
      for (int t0 = b0 + threadIdx.x; t0 < b1; t0 += 8 * kBlock) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = t0 + u * kBlock < b1 ? ea.e[t0 + u * kBlock] : 0.f;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (t0 + u * kBlock < b1) acc += (double)v[u];
      }
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = red[0];
    if (!isfinite(v)) atomicOr(ea.status, kStatusNonFinite);
    ea.out[sys] = ea.accumulate ? ea.out[sys] + v : v;
  }
}

// F_atom += self + sum over the atom's radial list entries (FP64): 16 lanes
// per atom, each summing a strided part of the row, then a shuffle tree.
// With `assign` the sum overwrites F_atom (every row of the output is an NNP
// atom and the call does not accumulate), which saves clearing it first.
// Blocks from gather_blocks on reduce the energies instead.
__global__ __launch_bounds__(kBlock) void k_force_gather(const float3* __restrict__ contrib,
                                                         const double* __restrict__ self,
                                                         const int* __restrict__ rad_off,
                                                         const int* __restrict__ slot_atom, int n, int S,
                                                         int max_rad, double* __restrict__ forces,
                                                         double* __restrict__ link_forces, int assign,
                                                         int gather_blocks, EnergyArgs ea) {
  // the energy blocks come first, so that their serial reduction runs beside
  // the gather instead of after it
  const int energy_blocks = (int)gridDim.x - gather_blocks;
  if ((int)blockIdx.x < energy_blocks) {
    energy_block(ea, (int)blockIdx.x);
    return;
  }
  const int gid = ((int)blockIdx.x - energy_blocks) * blockDim.x + threadIdx.x;
  const int i = gid >> 4;
  const int sub = gid & 15;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (i < n) {
    const int nr = rad_off[(int64_t)i * (S + 1) + S];
    const float3* row = contrib + (int64_t)i * max_rad;   // 16 lanes read 192 contiguous bytes
    for (int t = sub; t < nr; t += 16) {
      const float3 v = row[t];
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
    fx += self[3 * (int64_t)i];
    fy += self[3 * (int64_t)i + 1];
    fz += self[3 * (int64_t)i + 2];
    if (!assign) {
      fx += f[0];
      fy += f[1];
      fz += f[2];
    }
    f[0] = fx;
    f[1] = fy;
    f[2] = fz;
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

// Forward descriptor variants: 0 = one wavefront per atom, 1 = one 16-lane
// row per atom (default), 2 = one 8-lane row per atom (fewer idle lanes,
// half the wavefronts: for large systems), 3 and 4 = the pool kernel with two
// and four atoms per wavefront (many elements: few pairs per class).
int descriptor_variant(const nnp_model& m, int n) {
  const int v = stage_variant(m, kTuneDescriptor, n);
  return v >= 0 ? v : 1;
}

hipError_t launch_descriptor_fwd(nnp_model& m, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  FwdArgs a;
  a.order = m.d_order;
  a.spos = m.d_spos;
  a.rad = m.d_nbr_rad;
  a.ang = m.d_nbr_ang;
  a.rad_off = m.d_rad_off;
  a.ang_off = m.d_ang_off;
  a.max_rad = m.max_rad;
  a.max_ang = m.max_ang;
  a.n = n;
  a.x = m.d_x;
  const int v = descriptor_variant(m, n);
  if (v == 3 || v == 4) {
    const int aw = v == 3 ? 2 : 4;
    const size_t area = (std::max((size_t)aw * m.max_ang * 5, (size_t)64 * kPoolPitch) + 3) & ~(size_t)3;
    const size_t lds = 4 * sizeof(float) * (area + 64);   // four wavefronts, each with its own slice
    const unsigned blocks = (unsigned)((n + 4 * aw - 1) / (4 * aw));
    if (v == 3)
      hipLaunchKernelGGL(k_desc_fwd_pool<2>, dim3(blocks), dim3(256), lds, st, a, m.dp, m.geo);
    else
      hipLaunchKernelGGL(k_desc_fwd_pool<4>, dim3(blocks), dim3(256), lds, st, a, m.dp, m.geo);
  } else if (v == 1) {
    const size_t lds = (sizeof(float4) + sizeof(float)) * 16 * (size_t)m.max_ang;
    hipLaunchKernelGGL(k_desc_fwd_rows<16>, dim3((n + 15) / 16), dim3(256), lds, st, a, m.dp, m.geo);
  } else if (v == 2) {
    const size_t lds = (sizeof(float4) + sizeof(float)) * 32 * (size_t)m.max_ang;
    hipLaunchKernelGGL(k_desc_fwd_rows<8>, dim3((n + 31) / 32), dim3(256), lds, st, a, m.dp, m.geo);
  } else {
    const size_t lds = sizeof(float) * (64 * (size_t)kPartStride + 5 * (size_t)m.max_ang);
    hipLaunchKernelGGL(k_desc_fwd, dim3(n), dim3(64), lds, st, a, m.dp, m.geo);
  }
  return hipGetLastError();
}

// Adjoint variants: 0 = one wavefront per atom (default; measured faster on
// water boxes), 1 = half a wavefront per atom, 2 = variant 0 with the wide
// reverse-slot count (for lists far beyond the caches).
int adjoint_variant(const nnp_model& m, int n) {
  const int v = stage_variant(m, kTuneAdjoint, n);
  return v >= 0 ? v : 0;
}

hipError_t launch_descriptor_bwd(nnp_model& m, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  BwdArgs a;
  a.order = m.d_order;
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
  const size_t per_atom = bwd_lds_per_atom(m.max_rad, m.max_ang, m.stride);
  const int v = adjoint_variant(m, n);
  if (v == 1) {
    hipLaunchKernelGGL((k_desc_bwd<32, false>), dim3((n + 1) / 2), dim3(64), 2 * per_atom, st, a, m.dp, m.geo);
  } else if (v == 2) {
    hipLaunchKernelGGL((k_desc_bwd<64, true>), dim3(n), dim3(64), per_atom, st, a, m.dp, m.geo);
  } else {
    hipLaunchKernelGGL((k_desc_bwd<64, false>), dim3(n), dim3(64), per_atom, st, a, m.dp, m.geo);
  }
  return hipGetLastError();
}

hipError_t launch_force_gather(nnp_model& m, int n, double* forces, int assign, double* energies, int n_sys,
                               int accumulate, hipStream_t st) {
  EnergyArgs ea;
  const bool single = m.geo.periodic || m.geo.n_bins == 1;
  ea.part = single ? m.d_part : nullptr;
  ea.e = m.d_e;
  ea.bin_start = m.d_bin_start;
  ea.n_bins = m.geo.n_bins;
  ea.S = m.S;
  ea.tile_rows = 16 * m.mlp_cols;
  ea.mixed = m.mlp_mixed;
  ea.empty = n == 0;
  ea.out = energies;
  ea.accumulate = accumulate;
  ea.status = m.d_status;
  const int gather_blocks = (int)((16 * (int64_t)n + kBlock - 1) / kBlock);
  const int energy_blocks = single ? 1 : n_sys;
  hipLaunchKernelGGL(k_force_gather, dim3((unsigned)(gather_blocks + energy_blocks)), dim3(kBlock), 0, st,
                     m.d_contrib, m.d_self, m.d_rad_off, m.d_slot_atom, n, m.S, m.max_rad, forces, m.d_link_F,
                     assign, gather_blocks, ea);
  return hipGetLastError();
}

}  // namespace nnp
