// Per-element networks on the matrix cores: forward (atomic energies, whose
// sum is E_ML of Theory, eq. 1) and the hand-written backward (dE/d
// descriptor, the first link of eq. 2), fused in one kernel.
//
// Layout trick.  Each wavefront owns 16 atoms of one species and computes the
// TRANSPOSED products  H_l^T [features x 16 atoms] = W_l [out x in] * H_{l-1}^T,
// so the weights are the A operand and the activations the B operand of
// v_mfma_f32_16x16x{4f32,32_bf16}.  The accumulator layout of one 16x16
// output tile (lane = atom + 16 q holds features 4q..4q+3) is exactly the B
// operand layout the next layer needs for a 16-wide (FP32) or, taking two
// tiles, 32-wide (BF16) K block, provided the K dimension is permuted the same
// way in the packed weights.  The whole chain -- three hidden layers, the
// output layer, and the three backward products -- therefore stays in
// registers: no LDS, no barriers.  Weights are pre-packed on the host in
// fragment order (one 16-byte load per lane per MFMA step).
//
// Backward: e = w4 . h3 + b4, delta3 = w4 o celu'(u3), delta2 = (W3^T delta3) o
// celu'(u2), delta1 = (W2^T delta2) o celu'(u1), dE/dx = W1^T delta1, with
// celu'(u) recovered from h = celu(u): 1 for h > 0, else h/alpha + 1.
// An ensemble averages e and dE/dx over its members.
#include <type_traits>

#include "nnp_internal.h"

namespace nnp {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ v4f mfma_step(const v4f& w, const v4f& b, v4f c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(w[0], b[0], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(w[1], b[1], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(w[2], b[2], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(w[3], b[3], c, 0, 0, 0);
  return c;
}

__device__ __forceinline__ v8bf to_bf16x8(const v4f& lo, const v4f& hi) {
  v8bf r;
  r[0] = (__bf16)lo[0]; r[1] = (__bf16)lo[1]; r[2] = (__bf16)lo[2]; r[3] = (__bf16)lo[3];
  r[4] = (__bf16)hi[0]; r[5] = (__bf16)hi[1]; r[6] = (__bf16)hi[2]; r[7] = (__bf16)hi[3];
  return r;
}

__device__ __forceinline__ v4bf to_bf16x4(const v4f& v) {
  v4bf r;
  r[0] = (__bf16)v[0]; r[1] = (__bf16)v[1]; r[2] = (__bf16)v[2]; r[3] = (__bf16)v[3];
  return r;
}

// Weight fragments are streamed from L2 with a prefetch ring: the loads for
// K block kb + kPrefetch are issued before the products of block kb, so
// several fragment loads are in flight behind the matrix-core work.  (The
// wide H/C/N/O networks keep a shallower ring to stay clear of spills.)
// A BF16 step is an eighth of an FP32 step's matrix-core time, so its ring is
// deeper.
template <bool BF16, bool WIDE>
struct PrefetchDepth {
  static constexpr int value = WIDE ? (BF16 ? 3 : 2) : (BF16 ? 6 : 3);
};

template <bool BF16>
struct Frag {
  using T = v4f;
};
template <>
struct Frag<true> {
  using T = v8bf;
};

__device__ __forceinline__ v4f mma(const v4f& w, const v4f& b, v4f c) { return mfma_step(w, b, c); }
__device__ __forceinline__ v4f mma(const v8bf& w, const v8bf& b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, b, c, 0, 0, 0);
}

// out[R/16 tiles] (+)= W[R x C] * in[C/16 tiles]; `in` is register resident.
// Row tiles are processed in chunks of CH to bound the live accumulators.
template <int R, int C, bool BF16, int CH>
__device__ __forceinline__ void gemm_regs(const void* __restrict__ W, const v4f* in, v4f* out, int lane) {
  static_assert(R % 16 == 0 && C % (BF16 ? 32 : 16) == 0, "tile sizes");
  constexpr int kPrefetch = PrefetchDepth<BF16, (R > 160 || C > 160)>::value;
  constexpr int RT = R / 16;
  constexpr int KB = BF16 ? C / 32 : C / 16;
  using F = typename Frag<BF16>::T;
  const F* Wp = reinterpret_cast<const F*>(W);
#pragma unroll
  for (int r0 = 0; r0 < RT; r0 += CH) {
    const int nr = (r0 + CH < RT ? CH : RT - r0);
    F ring[kPrefetch][CH];
#pragma unroll
    for (int p = 0; p < kPrefetch; ++p)
#pragma unroll
      for (int r = 0; r < CH; ++r)
        if (p < KB && r < nr) ring[p][r] = Wp[((r0 + r) * KB + p) * 64 + lane];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      F cur[CH];
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        cur[r] = ring[kb % kPrefetch][r];
        if (kb + kPrefetch < KB && r < nr) ring[kb % kPrefetch][r] = Wp[((r0 + r) * KB + kb + kPrefetch) * 64 + lane];
      }
      if constexpr (BF16) {
        const v8bf b = to_bf16x8(in[2 * kb], in[2 * kb + 1]);
#pragma unroll
        for (int r = 0; r < CH; ++r)
          if (r < nr) out[r0 + r] = mma(cur[r], b, out[r0 + r]);
      } else {
#pragma unroll
        for (int r = 0; r < CH; ++r)
          if (r < nr) out[r0 + r] = mma(cur[r], in[kb], out[r0 + r]);
      }
    }
  }
}

__device__ __forceinline__ float celu_f(float u, float alpha, float inv_alpha_l2) {
  return u > 0.f ? u : alpha * (__builtin_amdgcn_exp2f(u * inv_alpha_l2) - 1.f);
}
__device__ __forceinline__ float celu_grad_from_h(float h, float inv_alpha) {
  return h > 0.f ? 1.f : h * inv_alpha + 1.f;
}

// Packed per-(member, species) layout of the matrices, in elements:
//   F1 [N1 x K0], F2 [N2 x N1], F3 [N3 x N2]   forward,  A = W_l
//   B1 [K0 x N1], B2 [N1 x N2], B3 [N2 x N3]   backward, A = W_l^T
// and of the vectors (FP32): b1[N1] b2[N2] b3[N3] w4[N3] b4[4].
//
// One workgroup (4 wavefronts) owns a tile of 16*C atoms of one species.
// Every product is split by output row tiles: wavefront w computes the row
// tiles r = w, w+4, ... for all C column tiles (each weight fragment it loads
// serves C matrix-core steps) and publishes them in LDS, in the same fragment
// layout, for the next product.  Each wavefront keeps its own post-activation
// tiles in registers for the CELU derivative of the backward pass.
template <int R, int NW>
struct Own {  // number of row tiles r = w + NW j owned by one of NW wavefronts
  static constexpr int n = (R + NW - 1) / NW;
};

// Layer outputs in LDS, per column tile c and row tile r (16 features):
//   FP32: one v4f per lane at [(c * tiles + r) * 64 + lane];
//   BF16: rounded once by the producer, two row tiles form the 16-byte B
//     fragment of one 32-wide K block, [(c * tiles/2 + r/2) * 64 + lane],
//     row tile r filling half r % 2 (the K permutation of the packed weights).
template <bool BF16>
__device__ __forceinline__ void put_tile(v4f* buf, int tiles, int c, int r, int lane, const v4f& v) {
  if constexpr (BF16)
    reinterpret_cast<v4bf*>(buf)[((c * (tiles / 2) + (r >> 1)) * 64 + lane) * 2 + (r & 1)] = to_bf16x4(v);
  else
    buf[(c * tiles + r) * 64 + lane] = v;
}

// out[j][c] = A-rows (w + 4 j) of W [R x K] times the K/16 LDS tiles `in[c][kb]`.
template <int R, int K, bool BF16, int C, int NW>
__device__ __forceinline__ void gemm_lds(const void* __restrict__ W, const v4f* in, int in_tiles, v4f (*out)[C],
                                         int w, int lane, int cw) {
  constexpr int NJ = Own<R, NW>::n;
  constexpr int KB = BF16 ? K / 32 : K / 16;
  constexpr int kPrefetch = PrefetchDepth<BF16, (16 * R > 160 || K > 160)>::value;
  using F = typename Frag<BF16>::T;
  const F* Wp = reinterpret_cast<const F*>(W);
  F ring[kPrefetch][NJ];
#pragma unroll
  for (int p = 0; p < kPrefetch; ++p)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int r = w + NW * j;
      if (p < KB && r < R) ring[p][j] = Wp[(r * KB + p) * 64 + lane];
    }
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    F cur[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int r = w + NW * j;
      cur[j] = ring[kb % kPrefetch][j];
      if (kb + kPrefetch < KB && r < R) ring[kb % kPrefetch][j] = Wp[(r * KB + kb + kPrefetch) * 64 + lane];
    }
    F bv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (c >= cw) continue;   // a narrow tile (workgroup-uniform)
      if constexpr (BF16)
        bv[c] = reinterpret_cast<const v8bf*>(in)[(c * (in_tiles / 2) + kb) * 64 + lane];
      else
        bv[c] = in[(c * in_tiles + kb) * 64 + lane];
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int r = w + NW * j;
      if (r < R) {
#pragma unroll
        for (int c = 0; c < C; ++c)
          if (c < cw) out[j][c] = mma(cur[j], bv[c], out[j][c]);
      }
    }
  }
}

// CHG: the network has a second output, an atomic charge q_i in the MM
// potential phi_i (input column phi_col): the atomic energy is e_i + q_i phi_i,
// the backward seed of the last hidden layer is (w_e + phi_i w_q), and q_i is
// written out for the MM adjoint (dE/dphi_i gets the direct term q_i).
template <int K0, int N1, int N2, int N3, bool BF16, int C, bool MIXED, int NW, bool CHG>
__device__ __forceinline__ void mlp_split_body(const MlpArgs& a, float alpha) {
  constexpr int oF1 = 0, oF2 = oF1 + N1 * K0, oF3 = oF2 + N2 * N1;
  constexpr int oB1 = oF3 + N3 * N2, oB2 = oB1 + K0 * N1, oB3 = oB2 + N1 * N2;
  constexpr int ob1 = 0, ob2 = ob1 + N1, ob3 = ob2 + N2, ow4 = ob3 + N3, ob4 = ow4 + N3;
  constexpr int owq = ob4 + 4, obq = owq + N3;   // charge row (CHG)
  constexpr int TX = (K0 > N2 ? K0 : N2) / 16;        // tiles of buffer X (x, then H2, then delta2)
  constexpr int TA = (N1 > N3 ? N1 : N3) / 16;        // tiles of buffer A (H1, then delta3, then delta1)
  using Elem = typename std::conditional<BF16, __bf16, float>::type;
  __shared__ v4f bufX[C * TX * (BF16 ? 32 : 64)];   // BF16 tiles take half the space
  __shared__ v4f bufA[C * TA * (BF16 ? 32 : 64)];
  __shared__ float epart[NW][C * 16];
  __shared__ float qpart[CHG ? NW : 1][C * 16];

  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4;
  const int col = lane & 15;

  // workgroup -> (species, tile of 16*cw rows); cw = C except for the narrow
  // species of the mixed tiling
  const int narrow = MIXED ? narrow_species(a.bin_start, a.S, a.n_bins) : -1;
  int s = -1, row0 = 0, row_end = 0, before = 0, cw = C;
  for (int ss = 0; ss < a.S; ++ss) {
    const int b0 = a.bin_start[ss * a.n_bins], b1 = a.bin_start[(ss + 1) * a.n_bins];
    const int width = ss == narrow ? 1 : C;
    const int nt = (b1 - b0 + 16 * width - 1) / (16 * width);
    if ((int)blockIdx.x < before + nt) {
      s = ss;
      cw = width;
      row0 = b0 + ((int)blockIdx.x - before) * 16 * width;
      row_end = min(b1, row0 + 16 * width);
      break;
    }
    before += nt;
  }
  if (s < 0) return;   // whole workgroup exits together
  const float inv_alpha = 1.f / alpha;
  const float inv_alpha_l2 = kLog2e / alpha;

  float e_acc[C], q_acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) e_acc[c] = q_acc[c] = 0.f;
  float phi[C];   // MM potential of each column's atom (CHG)
#pragma unroll
  for (int c = 0; c < C; ++c) {
    phi[c] = 0.f;
    if constexpr (CHG) {
      const int row = row0 + c * 16 + col;
      if (row < row_end) phi[c] = a.x[(int64_t)row * a.stride + a.phi_col];
    }
  }

  for (int mem = 0; mem < a.n_members; ++mem) {
    const Elem* Wm = reinterpret_cast<const Elem*>(a.wmat) + (int64_t)(mem * a.S + s) * a.mat_per_species;
    const float* V = a.wvec + (int64_t)(mem * a.S + s) * a.vec_per_species;

    // stage x in fragment layout (again for every member: the buffer is reused
    // by later products): tile (c, kb), lane l holds x[row c*16 + l%16][16 kb + 4 (l/16) .. +3]
    if constexpr (BF16) {   // K block kb of 32 features: tiles 2 kb and 2 kb + 1
      for (int t = threadIdx.x; t < C * (K0 / 32) * 64; t += 64 * NW) {
        const int l = t & 63, kb = (t >> 6) % (K0 / 32), c = (t >> 6) / (K0 / 32);
        const int row = row0 + c * 16 + (l & 15);
        v4f lo = v4f{0.f, 0.f, 0.f, 0.f}, hi = lo;
        if (row < row_end) {
          const float* src = a.x + (int64_t)row * a.stride + 32 * kb + 4 * (l >> 4);
          lo = *reinterpret_cast<const v4f*>(src);
          hi = *reinterpret_cast<const v4f*>(src + 16);
        }
        reinterpret_cast<v8bf*>(bufX)[(c * (TX / 2) + kb) * 64 + l] = to_bf16x8(lo, hi);
      }
    } else {
      for (int t = threadIdx.x; t < C * (K0 / 16) * 64; t += 64 * NW) {
        const int l = t & 63, kb = (t >> 6) % (K0 / 16), c = (t >> 6) / (K0 / 16);
        const int row = row0 + c * 16 + (l & 15);
        v4f v = v4f{0.f, 0.f, 0.f, 0.f};
        if (row < row_end) v = *reinterpret_cast<const v4f*>(a.x + (int64_t)row * a.stride + 16 * kb + 4 * (l >> 4));
        bufX[(c * TX + kb) * 64 + l] = v;
      }
    }
    __syncthreads();

    // ---- layer 1: h1 = celu(W1 x + b1)       X -> A
    v4f h1[Own<N1, NW>::n][C];
#pragma unroll
    for (int j = 0; j < Own<N1, NW>::n; ++j) {
      const int r = w + NW * j;
      const v4f bias = r < N1 / 16 ? *reinterpret_cast<const v4f*>(V + ob1 + 16 * r + 4 * q) : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < C; ++c) h1[j][c] = bias;
    }
    gemm_lds<N1 / 16, K0, BF16, C, NW>(Wm + oF1, bufX, TX, h1, w, lane, cw);
#pragma unroll
    for (int j = 0; j < Own<N1, NW>::n; ++j) {
      const int r = w + NW * j;
      if (r < N1 / 16) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
          for (int t = 0; t < 4; ++t) h1[j][c][t] = celu_f(h1[j][c][t], alpha, inv_alpha_l2);
          put_tile<BF16>(bufA, TA, c, r, lane, h1[j][c]);
        }
      }
    }
    __syncthreads();

    // ---- layer 2: h2 = celu(W2 h1 + b2)      A -> X
    v4f h2[Own<N2, NW>::n][C];
#pragma unroll
    for (int j = 0; j < Own<N2, NW>::n; ++j) {
      const int r = w + NW * j;
      const v4f bias = r < N2 / 16 ? *reinterpret_cast<const v4f*>(V + ob2 + 16 * r + 4 * q) : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < C; ++c) h2[j][c] = bias;
    }
    gemm_lds<N2 / 16, N1, BF16, C, NW>(Wm + oF2, bufA, TA, h2, w, lane, cw);
    __syncthreads();   // everyone has read A (h1) and X (x) before X is overwritten
#pragma unroll
    for (int j = 0; j < Own<N2, NW>::n; ++j) {
      const int r = w + NW * j;
      if (r < N2 / 16) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
          for (int t = 0; t < 4; ++t) h2[j][c][t] = celu_f(h2[j][c][t], alpha, inv_alpha_l2);
          put_tile<BF16>(bufX, TX, c, r, lane, h2[j][c]);
        }
      }
    }
    __syncthreads();

    // ---- layer 3 and the output layer; delta3 = w4 o celu'(h3)   X -> A
    v4f h3[Own<N3, NW>::n][C];
#pragma unroll
    for (int j = 0; j < Own<N3, NW>::n; ++j) {
      const int r = w + NW * j;
      const v4f bias = r < N3 / 16 ? *reinterpret_cast<const v4f*>(V + ob3 + 16 * r + 4 * q) : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < C; ++c) h3[j][c] = bias;
    }
    gemm_lds<N3 / 16, N2, BF16, C, NW>(Wm + oF3, bufX, TX, h3, w, lane, cw);
    float ep[C];
    float eq[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ep[c] = eq[c] = 0.f;
#pragma unroll
    for (int j = 0; j < Own<N3, NW>::n; ++j) {
      const int r = w + NW * j;
      if (r < N3 / 16) {
        const v4f w4 = *reinterpret_cast<const v4f*>(V + ow4 + 16 * r + 4 * q);
        v4f wq = v4f{0.f, 0.f, 0.f, 0.f};
        if constexpr (CHG) wq = *reinterpret_cast<const v4f*>(V + owq + 16 * r + 4 * q);
#pragma unroll
        for (int c = 0; c < C; ++c) {
          v4f d;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const float h = celu_f(h3[j][c][t], alpha, inv_alpha_l2);
            ep[c] += w4[t] * h;
            if constexpr (CHG) {
              eq[c] += wq[t] * h;
              d[t] = fmaf(phi[c], wq[t], w4[t]) * celu_grad_from_h(h, inv_alpha);
            } else {
              d[t] = w4[t] * celu_grad_from_h(h, inv_alpha);
            }
          }
          put_tile<BF16>(bufA, TA, c, r, lane, d);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float v = ep[c];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (q == 0) epart[w][c * 16 + col] = v;
      if constexpr (CHG) {
        float u = eq[c];
        u += __shfl_xor(u, 16, 64);
        u += __shfl_xor(u, 32, 64);
        if (q == 0) qpart[w][c * 16 + col] = u;
      }
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c)
      {
        float e = 0.f;
#pragma unroll
        for (int u = 0; u < NW; ++u) e += epart[u][c * 16 + col];
        e += V[ob4];
        if constexpr (CHG) {
          float qa = 0.f;
#pragma unroll
          for (int u = 0; u < NW; ++u) qa += qpart[u][c * 16 + col];
          qa += V[obq];
          e = fmaf(qa, phi[c], e);
          q_acc[c] += qa;
        }
        e_acc[c] += e;
      }
    }

    // ---- delta2 = (W3^T delta3) o celu'(h2)    A -> X
    v4f d2[Own<N2, NW>::n][C];
#pragma unroll
    for (int j = 0; j < Own<N2, NW>::n; ++j)
#pragma unroll
      for (int c = 0; c < C; ++c) d2[j][c] = v4f{0.f, 0.f, 0.f, 0.f};
    gemm_lds<N2 / 16, N3, BF16, C, NW>(Wm + oB3, bufA, TA, d2, w, lane, cw);
#pragma unroll
    for (int j = 0; j < Own<N2, NW>::n; ++j) {
      const int r = w + NW * j;
      if (r < N2 / 16) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
          for (int t = 0; t < 4; ++t) d2[j][c][t] *= celu_grad_from_h(h2[j][c][t], inv_alpha);
          put_tile<BF16>(bufX, TX, c, r, lane, d2[j][c]);
        }
      }
    }
    __syncthreads();

    // ---- delta1 = (W2^T delta2) o celu'(h1)    X -> A
    v4f d1[Own<N1, NW>::n][C];
#pragma unroll
    for (int j = 0; j < Own<N1, NW>::n; ++j)
#pragma unroll
      for (int c = 0; c < C; ++c) d1[j][c] = v4f{0.f, 0.f, 0.f, 0.f};
    gemm_lds<N1 / 16, N2, BF16, C, NW>(Wm + oB2, bufX, TX, d1, w, lane, cw);
#pragma unroll
    for (int j = 0; j < Own<N1, NW>::n; ++j) {
      const int r = w + NW * j;
      if (r < N1 / 16) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
          for (int t = 0; t < 4; ++t) d1[j][c][t] *= celu_grad_from_h(h1[j][c][t], inv_alpha);
          put_tile<BF16>(bufA, TA, c, r, lane, d1[j][c]);
        }
      }
    }
    __syncthreads();

    // ---- dE/dx = W1^T delta1 (row tiles over the input features), to memory
    {
      v4f gx[Own<K0 / 16, NW>::n][C];
#pragma unroll
      for (int j = 0; j < Own<K0 / 16, NW>::n; ++j)
#pragma unroll
        for (int c = 0; c < C; ++c) gx[j][c] = v4f{0.f, 0.f, 0.f, 0.f};
      gemm_lds<K0 / 16, N1, BF16, C, NW>(Wm + oB1, bufA, TA, gx, w, lane, cw);
#pragma unroll
      for (int j = 0; j < Own<K0 / 16, NW>::n; ++j) {
        const int r = w + NW * j;
        if (r < K0 / 16) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const int row = row0 + c * 16 + col;
            if (row < row_end) {
              v4f* dst = reinterpret_cast<v4f*>(a.g + (int64_t)row * a.stride + 16 * r + 4 * q);
              v4f v = gx[j][c];
              if (a.n_members > 1) {
                if (mem > 0) v += *dst;
                if (mem == a.n_members - 1) v *= (1.f / (float)a.n_members);
              }
              *dst = v;
            }
          }
        }
      }
    }
    __syncthreads();   // buffers are reused by the next ensemble member
  }
  // atomic energies and the tile's FP64 partial sum
  if (w == 0) {
    double ev = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int row = row0 + c * 16 + col;
      const float e_atom = e_acc[c] / (float)a.n_members;
      if (row < row_end && q == 0) {
        a.e[row] = e_atom;
        if constexpr (CHG) a.q[row] = q_acc[c] / (float)a.n_members;
        ev += (double)e_atom;
      }
    }
    if (a.part != nullptr) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) ev += __shfl_xor(ev, off, 64);
      if (lane == 0) a.part[blockIdx.x] = ev;
    }
  }
}

template <int K0, int N1, int N2, int N3, bool BF16, int C>
__global__ __launch_bounds__(256, K0 <= 128 ? 2 : 1) void k_mlp_split(MlpArgs a, float alpha) {
  mlp_split_body<K0, N1, N2, N3, BF16, C, false, 4, false>(a, alpha);
}

// Eight wavefronts per 16-atom tile: each owns half as many row tiles of
// every product, so a tile's chain is shorter.  For systems with too few
// tiles to fill the GPU (a small ML region: a tile per species).
template <int K0, int N1, int N2, int N3, bool BF16, int C, bool MIXED>
__global__ __launch_bounds__(512) void k_mlp_split8(MlpArgs a, float alpha) {
  mlp_split_body<K0, N1, N2, N3, BF16, C, MIXED, 8, false>(a, alpha);
}

// Mixed tiling: tiles of 32 atoms, of 16 for the species with the fewest
// atoms.  For a small system the workgroups then come in two sizes whose
// count matches the CUs better than one size does (water, 4,096 molecules:
// 256 + 256 instead of 384 tiles).  Every atom's arithmetic is the same as
// in the uniform tiling.
template <int K0, int N1, int N2, int N3, bool BF16>
__global__ __launch_bounds__(256, K0 <= 128 ? 2 : 1) void k_mlp_mixed(MlpArgs a, float alpha) {
  mlp_split_body<K0, N1, N2, N3, BF16, 2, true, 4, false>(a, alpha);
}

// The same kernels for networks with the charge output (MM channel models).
template <int K0, int N1, int N2, int N3, bool BF16, int C, bool MIXED, int NW>
__global__ __launch_bounds__(64 * NW, 1) void k_mlp_split_q(MlpArgs a, float alpha) {
  mlp_split_body<K0, N1, N2, N3, BF16, C, MIXED, NW, true>(a, alpha);
}

// Register-resident variant: each wavefront owns 16 atoms and keeps the whole
// chain (activations and deltas) in registers; no LDS, no barriers.  Cheapest
// when the products are short (BF16 operands).
template <int K0, int N1, int N2, int N3, bool BF16>
__global__ __launch_bounds__(kBlock) void k_mlp_reg(MlpArgs a, float alpha) {
  constexpr int oF1 = 0, oF2 = oF1 + N1 * K0, oF3 = oF2 + N2 * N1;
  constexpr int oB1 = oF3 + N3 * N2, oB2 = oB1 + K0 * N1, oB3 = oB2 + N1 * N2;
  constexpr int ob1 = 0, ob2 = ob1 + N1, ob3 = ob2 + N2, ow4 = ob3 + N3, ob4 = ow4 + N3;
  using Elem = typename std::conditional<BF16, __bf16, float>::type;

  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;
  const int q = lane >> 4;

  // wave -> (species, 16-row tile) from the species bucket boundaries
  int s = -1, row0 = 0, row_end = 0, before = 0;
  for (int ss = 0; ss < a.S; ++ss) {
    int b0 = a.bin_start[ss * a.n_bins], b1 = a.bin_start[(ss + 1) * a.n_bins];
    int nt = (b1 - b0 + 15) >> 4;
    if (wave < before + nt) {
      s = ss;
      row0 = b0 + (wave - before) * 16;
      row_end = b1;
      break;
    }
    before += nt;
  }
  if (s < 0) return;
  const int row = row0 + col;
  const bool valid = row < row_end;
  const float inv_alpha = 1.f / alpha;
  const float inv_alpha_l2 = kLog2e / alpha;
  const float* xrow = a.x + (int64_t)row * a.stride;
  float* grow = a.g + (int64_t)row * a.stride;
  float e_sum = 0.f;

  for (int mem = 0; mem < a.n_members; ++mem) {
    const Elem* Wm = reinterpret_cast<const Elem*>(a.wmat) + (int64_t)(mem * a.S + s) * a.mat_per_species;
    const float* V = a.wvec + (int64_t)(mem * a.S + s) * a.vec_per_species;

    // ---- layer 1: h1 = celu(W1 x + b1); x streamed from memory
    v4f h1[N1 / 16];
#pragma unroll
    for (int r = 0; r < N1 / 16; ++r) h1[r] = *reinterpret_cast<const v4f*>(V + ob1 + 16 * r + 4 * q);
    if constexpr (!BF16) {
      const v4f* Wp = reinterpret_cast<const v4f*>(Wm + oF1);
#pragma unroll 2
      for (int kb = 0; kb < K0 / 16; ++kb) {
        v4f xb = valid ? *reinterpret_cast<const v4f*>(xrow + 16 * kb + 4 * q) : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < N1 / 16; ++r) h1[r] = mfma_step(Wp[(r * (K0 / 16) + kb) * 64 + lane], xb, h1[r]);
      }
    } else {
      const v8bf* Wp = reinterpret_cast<const v8bf*>(Wm + oF1);
#pragma unroll 2
      for (int kb = 0; kb < K0 / 32; ++kb) {
        v4f lo = v4f{0.f, 0.f, 0.f, 0.f}, hi = v4f{0.f, 0.f, 0.f, 0.f};
        if (valid) {
          lo = *reinterpret_cast<const v4f*>(xrow + 32 * kb + 4 * q);
          hi = *reinterpret_cast<const v4f*>(xrow + 32 * kb + 16 + 4 * q);
        }
        v8bf xb = to_bf16x8(lo, hi);
#pragma unroll
        for (int r = 0; r < N1 / 16; ++r)
          h1[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wp[(r * (K0 / 32) + kb) * 64 + lane], xb, h1[r], 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < N1 / 16; ++r)
#pragma unroll
      for (int t = 0; t < 4; ++t) h1[r][t] = celu_f(h1[r][t], alpha, inv_alpha_l2);

    // ---- layer 2
    v4f h2[N2 / 16];
#pragma unroll
    for (int r = 0; r < N2 / 16; ++r) h2[r] = *reinterpret_cast<const v4f*>(V + ob2 + 16 * r + 4 * q);
    gemm_regs<N2, N1, BF16, 4>(Wm + oF2, h1, h2, lane);
#pragma unroll
    for (int r = 0; r < N2 / 16; ++r)
#pragma unroll
      for (int t = 0; t < 4; ++t) h2[r][t] = celu_f(h2[r][t], alpha, inv_alpha_l2);

    // ---- layer 3
    v4f h3[N3 / 16];
#pragma unroll
    for (int r = 0; r < N3 / 16; ++r) h3[r] = *reinterpret_cast<const v4f*>(V + ob3 + 16 * r + 4 * q);
    gemm_regs<N3, N2, BF16, 4>(Wm + oF3, h2, h3, lane);
#pragma unroll
    for (int r = 0; r < N3 / 16; ++r)
#pragma unroll
      for (int t = 0; t < 4; ++t) h3[r][t] = celu_f(h3[r][t], alpha, inv_alpha_l2);

    // ---- output layer and delta3 (in place)
    float ep = 0.f;
#pragma unroll
    for (int r = 0; r < N3 / 16; ++r) {
      v4f w4 = *reinterpret_cast<const v4f*>(V + ow4 + 16 * r + 4 * q);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        ep += w4[t] * h3[r][t];
        h3[r][t] = w4[t] * celu_grad_from_h(h3[r][t], inv_alpha);
      }
    }
    ep += __shfl_xor(ep, 16, 64);
    ep += __shfl_xor(ep, 32, 64);
    e_sum += ep + V[ob4];

    // ---- delta2 = (W3^T delta3) o celu'(h2)
    v4f d2[N2 / 16];
#pragma unroll
    for (int r = 0; r < N2 / 16; ++r) d2[r] = v4f{0.f, 0.f, 0.f, 0.f};
    gemm_regs<N2, N3, BF16, 4>(Wm + oB3, h3, d2, lane);
#pragma unroll
    for (int r = 0; r < N2 / 16; ++r)
#pragma unroll
      for (int t = 0; t < 4; ++t) h2[r][t] = d2[r][t] * celu_grad_from_h(h2[r][t], inv_alpha);

    // ---- delta1 = (W2^T delta2) o celu'(h1)
    v4f d1[N1 / 16];
#pragma unroll
    for (int r = 0; r < N1 / 16; ++r) d1[r] = v4f{0.f, 0.f, 0.f, 0.f};
    gemm_regs<N1, N2, BF16, 4>(Wm + oB2, h2, d1, lane);
#pragma unroll
    for (int r = 0; r < N1 / 16; ++r)
#pragma unroll
      for (int t = 0; t < 4; ++t) h1[r][t] = d1[r][t] * celu_grad_from_h(h1[r][t], inv_alpha);

    // ---- dE/dx = W1^T delta1, in chunks of row tiles streamed to memory
    constexpr int CH = 8;
    constexpr int RT0 = K0 / 16;
#pragma unroll
    for (int r0 = 0; r0 < RT0; r0 += CH) {
      v4f gx[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) gx[c] = v4f{0.f, 0.f, 0.f, 0.f};
      if constexpr (!BF16) {
        const v4f* Wp = reinterpret_cast<const v4f*>(Wm + oB1);
#pragma unroll
        for (int kb = 0; kb < N1 / 16; ++kb)
#pragma unroll
          for (int c = 0; c < CH; ++c)
            if (r0 + c < RT0) gx[c] = mfma_step(Wp[((r0 + c) * (N1 / 16) + kb) * 64 + lane], h1[kb], gx[c]);
      } else {
        const v8bf* Wp = reinterpret_cast<const v8bf*>(Wm + oB1);
#pragma unroll
        for (int kb = 0; kb < N1 / 32; ++kb) {
          v8bf b = to_bf16x8(h1[2 * kb], h1[2 * kb + 1]);
#pragma unroll
          for (int c = 0; c < CH; ++c)
            if (r0 + c < RT0)
              gx[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Wp[((r0 + c) * (N1 / 32) + kb) * 64 + lane], b, gx[c], 0, 0, 0);
        }
      }
      if (valid) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          if (r0 + c < RT0) {
            v4f* dst = reinterpret_cast<v4f*>(grow + 16 * (r0 + c) + 4 * q);
            v4f v = gx[c];
            if (a.n_members > 1) {
              if (mem > 0) v += *dst;
              if (mem == a.n_members - 1) v *= (1.f / (float)a.n_members);
            }
            *dst = v;
          }
        }
      }
    }
  }
  const float e_atom = e_sum / (float)a.n_members;
  if (valid && q == 0) a.e[row] = e_atom;
  if (a.part != nullptr) {
    double ev = (valid && q == 0) ? (double)e_atom : 0.0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ev += __shfl_xor(ev, off, 64);
    if (lane == 0) a.part[wave] = ev;
  }
}

// ---------------------------------------------------------------------------
// BF16 network with the weights resident in LDS (water-sized networks).
//
// A persistent workgroup serves one species: it copies that species' W1, W2,
// W3 (BF16, row-major, about 115 KB with row padding) into LDS once, then
// every wavefront takes tiles of 16 or 32 atoms on its own and runs the whole
// fused chain -- three hidden layers, the output, and the three backward
// products -- with no barrier and no weight traffic beyond LDS.  Forward
// products read W fragments with two 8-byte LDS reads per lane; the backward
// products need W^T fragments of the same copy, which the gfx950 transposing
// read gives: within a group of 16 lanes, lane i's element j comes from
// position i % 4 of the 8-byte chunk addressed by lane 4 j + i / 4, so if
// lane 4 j + s addresses W[k0 + j][c0 + 4 s], lane i receives
// W[k0 .. k0 + 3][c0 + i]: four consecutive K values of column c0 + i, an A
// fragment of W^T.
// The activations needed again by the backward pass are kept as the BF16
// B fragments the next product reads anyway, so celu'(u) is taken from the
// BF16-rounded activation (h / alpha + 1 for h < 0, an absolute difference
// of at most 2^-9 from the FP32 activation's; the backward operands are
// rounded to BF16 in any case).
// Measured bounds (261,000 atoms): without the x loads and dE/dx stores the
// stage runs 18 % faster, without the elementwise CELU work 18 % faster,
// without the LDS weight reads no faster: the FP32 descriptor rows read and
// the FP32 dE/dx rows written (1 KB per atom) and the elementwise work limit
// it, not the matrix cores.
// Tilings of the LDS-resident kernel: C 16-atom column tiles per wavefront
// tile and NW wavefronts per workgroup (1 workgroup per CU: NW / 4
// wavefronts per SIMD).

// Row pitch in bytes of a BF16 matrix with `in` columns in LDS: the 16 rows
// of a forward fragment start in distinct bank pairs (pitch / 4 an odd
// multiple of 2, mod 32) and the transposing reads see at most two-way
// conflicts (pitch / 4 not 2 mod 32).
constexpr int lds_pitch(int in) {
  int p = 2 * in + 8;
  while (((p / 8) & 1) == 0 || (p / 4) % 32 == 2) p += 8;
  return p;
}

// The vectors come first, so that their reads use immediate offsets.
template <int K0, int N1, int N2, int N3>
struct LdsLayout {
  static constexpr int P1 = lds_pitch(K0), P2 = lds_pitch(N1), P3 = lds_pitch(N2);
  static constexpr int nvec = N1 + N2 + N3 + N3 + 4;   // b1 b2 b3 w4 b4 (FP32)
  static constexpr int vec = 0, w1 = (4 * nvec + 255) / 256 * 256, w2 = w1 + N1 * P1, w3 = w2 + N2 * P2;
  static constexpr int bytes = w3 + N3 * P3;
};

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) char lds_char;
typedef __attribute__((address_space(3))) v4s lds_v4s;

__device__ __forceinline__ v8bf join_bf16(v4s lo, v4s hi) {
  typedef short v8s __attribute__((ext_vector_type(8)));
  v8s r;
  r[0] = lo[0]; r[1] = lo[1]; r[2] = lo[2]; r[3] = lo[3];
  r[4] = hi[0]; r[5] = hi[1]; r[6] = hi[2]; r[7] = hi[3];
  return __builtin_bit_cast(v8bf, r);
}

// The LDS address is hidden from the optimizer so that it stays one register
// per product and every fragment read of the product is that register plus
// an immediate offset (LDS offsets beyond 64 KB do not fit the immediate, and
// the compiler would otherwise keep a separate address per fragment).
__device__ __forceinline__ const lds_char* opaque_lds(const lds_char* p) {
  asm volatile("" : "+v"(p));
  return p;
}

// Per-lane base of the fragments of W (forward: row 16 rt + lane % 16, K
// offset 4 (lane / 16)) or of W^T (transposed reads: lane 16 g + 4 j + s
// addresses W[4 g + j][4 s] of each 32 x 16 block).
template <int P, bool TRANS>
__device__ __forceinline__ const lds_char* frag_base(const lds_char* W, int lane) {
  if (TRANS) return opaque_lds(W + (4 * (lane >> 4) + ((lane >> 2) & 3)) * P + 8 * (lane & 3));
  return opaque_lds(W + (lane & 15) * P + 8 * (lane >> 4));
}

// A fragment of W (rows = outputs, row tile rt; K block kb over the inputs),
// or with TRANS of W^T (rows = inputs of W, row tile rt; K block kb over the
// outputs of W), from the per-lane base.
template <int P, bool TRANS>
__device__ __forceinline__ v8bf frag_at(const lds_char* base, int rt, int kb) {
  if (TRANS) {
    const lds_char* p0 = base + 32 * kb * P + 32 * rt;
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(p0));
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(p0 + 16 * P));
    return join_bf16(lo, hi);
  }
  const lds_char* row = base + 16 * rt * P + 64 * kb;
  return join_bf16(*(const lds_v4s*)(row), *(const lds_v4s*)(row + 32));
}

// One product, op(W) [R x K] times the B fragments [K/32][C], in chunks of CH
// row tiles (CH even): init(r0, acc) seeds a chunk's accumulators, the K
// blocks follow -- each block's fragments are read, then multiplied, with a
// compiler barrier between blocks so that the scheduler does not hoist every
// read of the product ahead of the matrix-core work (which would need
// registers for all of them at once) -- and epi(r0, acc) consumes the chunk
// (activation, conversion to the next product's B fragments, or the store).
// Only one chunk of accumulators is live.  (Reading the next block's
// fragments one step ahead was measured no faster.)
template <int R, int K, int P, bool TRANS, int CH, int C, typename Init, typename Epi>
__device__ __forceinline__ void lds_product(const lds_char* W, const v8bf (*B)[C], int lane, Init init, Epi epi) {
  static_assert(CH % 2 == 0, "chunks of whole K blocks of the next product");
  const lds_char* base = frag_base<P, TRANS>(W, lane);
#pragma unroll
  for (int r0 = 0; r0 < R / 16; r0 += CH) {
    v4f acc[CH][C];
    init(r0, acc);
#pragma unroll
    for (int kb = 0; kb < K / 32; ++kb) {
      v8bf A[CH];
#pragma unroll
      for (int r = 0; r < CH; ++r)
        if (r0 + r < R / 16) A[r] = frag_at<P, TRANS>(base, r0 + r, kb);
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        if (r0 + r < R / 16) {
#pragma unroll
          for (int c = 0; c < C; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[r], B[kb][c], acc[r][c], 0, 0, 0);
        }
      }
      asm volatile("" ::: "memory");
    }
    epi(r0, acc);
  }
}

// Accumulator tiles r0 .. r0 + CH - 1 (row tile rt: features 16 rt + 4 q + t)
// into the BF16 B fragments of the next product (K block rt / 2, element
// 4 (rt % 2) + t).
// The packed fragment is hidden from the optimizer: later reads of single
// elements (celu' in the backward pass) then come from the packed BF16
// registers, instead of the compiler keeping the FP32 values alive as well.
template <int R, int CH, int C>
__device__ __forceinline__ void chunk_to_frags(int r0, const v4f (*acc)[C], v8bf (*f)[C]) {
#pragma unroll
  for (int r = 0; r < CH; r += 2)
    if (r0 + r < R / 16)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        v8bf v = to_bf16x8(acc[r][c], acc[r + 1][c]);
        asm volatile("" : "+v"(v));
        f[(r0 + r) / 2][c] = v;
      }
}

// CELU in the form the kernel evaluates it: t = 2^(u log2(e) / alpha) and
// h = med3(u, alpha t - alpha, 0), since 0 < u < alpha (t - 1) for u > 0 and
// u <= alpha (t - 1) <= 0 for u <= 0 (near u = 0, where rounding can swap
// the order of the first two, either is returned; they then differ by about
// alpha 2^-23); its derivative is min(t, 1) (t > 1 exactly when u > 0), kept
// for the backward pass as packed FP16 (rounded toward zero: relative error
// below 2^-10).
__device__ __forceinline__ float celu_med3(float u, float t, float alpha) {
  return __builtin_amdgcn_fmed3f(u, fmaf(alpha, t, -alpha), 0.f);
}
// celu' from the activation h (the output layer's, in FP32): 1 for h > 0,
// else h / alpha + 1 = min(h / alpha + 1, 1) (h / alpha + 1 > 1 exactly when
// h > 0).
__device__ __forceinline__ float celu_grad_lean(float h, float inv_alpha) {
  return fminf(fmaf(h, inv_alpha, 1.f), 1.f);
}
__device__ __forceinline__ uint32_t celu_grad_pk(float t0, float t1) {
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(fminf(t0, 1.f), fminf(t1, 1.f)));
}
// x times the FP16 value in the low (HI false) or high half of d, rounded
// once.  It is written as fma(x, d, +0), which the compiler must keep as an
// fma (a zero product's sign can differ from the fma's) and emits as one
// mixed-precision fma instead of a conversion and a product, inserting
// itself the wait states after the matrix-core products whose results it
// reads.
template <bool HI>
__device__ __forceinline__ float mul_f16(float x, uint32_t d) {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  const h2 v = __builtin_bit_cast(h2, d);
  return __builtin_fmaf(x, (float)v[HI ? 1 : 0], 0.f);
}

// The FP16 derivatives of accumulator tiles r0 .. r0 + CH - 1 in the element
// order of chunk_to_frags: fragment rt / 2, dword 2 (rt % 2) + u / 2, half
// u % 2 for feature 16 rt + 4 q + u.
template <int R, int CH, int C>
__device__ __forceinline__ void chunk_to_grads(int r0, const v4f (*t)[C], uint32_t (*d)[C][4]) {
#pragma unroll
  for (int r = 0; r < CH; r += 2)
    if (r0 + r < R / 16)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        uint32_t* o = d[(r0 + r) / 2][c];
        o[0] = celu_grad_pk(t[r][c][0], t[r][c][1]);
        o[1] = celu_grad_pk(t[r][c][2], t[r][c][3]);
        o[2] = celu_grad_pk(t[r + 1][c][0], t[r + 1][c][1]);
        o[3] = celu_grad_pk(t[r + 1][c][2], t[r + 1][c][3]);
        asm volatile("" : "+v"(o[0]), "+v"(o[1]), "+v"(o[2]), "+v"(o[3]));
      }
}

template <int K0, int N1, int N2, int N3, int C, int NW>
__global__ __launch_bounds__(64 * NW, 1) void k_mlp_lds(MlpArgs a, float alpha) {
  using Lay = LdsLayout<K0, N1, N2, N3>;
  static_assert(K0 % 32 == 0 && N1 % 32 == 0 && N2 % 32 == 0 && N3 % 32 == 0, "32-wide K blocks");
  constexpr int CH = C == 1 ? 2 : 4;   // row tiles per accumulator chunk
  constexpr int TILE = 16 * C;
  __shared__ __attribute__((aligned(16))) char lds[Lay::bytes];
  const lds_char* L = (const lds_char*)lds;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4;
  const int col = lane & 15;

  // workgroup -> species: one workgroup per species with atoms, the rest in
  // proportion to the species' tiles; workgroups beyond them exit
  int T = 0, ne = 0;
  for (int s = 0; s < a.S; ++s) {
    const int ns = a.bin_start[(s + 1) * a.n_bins] - a.bin_start[s * a.n_bins];
    const int ts = (ns + TILE - 1) / TILE;
    T += ts;
    ne += ts > 0;
  }
  if (T == 0) return;
  const int G = (int)gridDim.x;
  int s_mine = -1, wg0 = 0, gs = 0, tiles_before = 0, ts_mine = 0, b0_mine = 0, b1_mine = 0;
  {
    int first = 0, tb = 0;
    for (int s = 0; s < a.S; ++s) {
      const int b0 = a.bin_start[s * a.n_bins], b1 = a.bin_start[(s + 1) * a.n_bins];
      const int ts = (b1 - b0 + TILE - 1) / TILE;
      const int g = ts > 0 ? 1 + (G - ne) * ts / T : 0;
      if ((int)blockIdx.x >= first && (int)blockIdx.x < first + g) {
        s_mine = s;
        wg0 = first;
        gs = g;
        tiles_before = tb;
        ts_mine = ts;
        b0_mine = b0;
        b1_mine = b1;
      }
      first += g;
      tb += ts;
    }
  }
  if (s_mine < 0) return;   // whole workgroup exits together

  // weights of the species into LDS: 16-byte pieces, eight loads in flight per
  // thread before their stores; vectors as FP32
  {
    const uint16_t* src = reinterpret_cast<const uint16_t*>(a.wrow) + (int64_t)s_mine * a.wrow_per_species;
    auto copy = [&](const uint16_t* m, int rows, int in, int pitch, int dst) {
      const int per_row = in / 8;
      const int total = rows * per_row;
      for (int t0 = threadIdx.x; t0 < total; t0 += 8 * 64 * NW) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = t0 + u * 64 * NW;
          if (t < total) {
            const int r = t / per_row, c = t - r * per_row;
            v[u] = *reinterpret_cast<const uint4*>(m + (int64_t)r * in + 8 * c);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int t = t0 + u * 64 * NW;
          if (t < total) {
            const int r = t / per_row, c = t - r * per_row;
            // the pitch is a multiple of 8 bytes only: two 8-byte stores
            uint2* d = reinterpret_cast<uint2*>(lds + dst + r * pitch + 16 * c);
            d[0] = make_uint2(v[u].x, v[u].y);
            d[1] = make_uint2(v[u].z, v[u].w);
          }
        }
      }
    };
    copy(src, N1, K0, Lay::P1, Lay::w1);
    copy(src + N1 * K0, N2, N1, Lay::P2, Lay::w2);
    copy(src + N1 * K0 + N2 * N1, N3, N2, Lay::P3, Lay::w3);
    const float* V = a.wvec + (int64_t)s_mine * a.vec_per_species;
    float* vl = reinterpret_cast<float*>(lds + Lay::vec);
    for (int t = threadIdx.x; t < Lay::nvec; t += 64 * NW) vl[t] = V[t];
  }
  __syncthreads();
  const lds_char* W1 = L + Lay::w1;
  const lds_char* W2 = L + Lay::w2;
  const lds_char* W3 = L + Lay::w3;
  const float* vb1 = reinterpret_cast<const float*>(lds + Lay::vec);
  const float* vb2 = vb1 + N1;
  const float* vb3 = vb2 + N2;
  const float* vw4 = vb3 + N3;
  const float b4 = vw4[N3];
  const float inv_alpha = 1.f / alpha;
  const float inv_alpha_l2 = kLog2e / alpha;
  const v4f zero = v4f{0.f, 0.f, 0.f, 0.f};

  const int waves = gs * NW;
  // tile t = rank * gs + workgroup, rank = wavefront in its workgroup: every
  // round of `waves` tiles gives each workgroup the same number, and a last,
  // partial round gives its tiles to the low ranks of every workgroup, which
  // fall on different SIMDs
  for (int t = w * gs + ((int)blockIdx.x - wg0); t < ts_mine; t += waves) {
    const int row0 = b0_mine + t * TILE;
    // x as B fragments: column tile c, K block kb: atom row0 + 16 c + col,
    // features 32 kb + 4 q .. +3 and 32 kb + 16 + 4 q .. +3 (zero beyond the
    // species)
    v8bf xf[K0 / 32][C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int row = row0 + 16 * c + col;
      const bool ok = row < b1_mine;
      const float* xr = a.x + (int64_t)(ok ? row : b0_mine) * a.stride + 4 * q;
#pragma unroll
      for (int kb = 0; kb < K0 / 32; ++kb) {
        v4f lo = *reinterpret_cast<const v4f*>(xr + 32 * kb);
        v4f hi = *reinterpret_cast<const v4f*>(xr + 32 * kb + 16);
        if (!ok) lo = hi = zero;
        xf[kb][c] = to_bf16x8(lo, hi);
      }
    }
    auto bias_init = [&](const float* b) {
      return [=](int r0, v4f (*acc)[C]) {
#pragma unroll
        for (int r = 0; r < CH; ++r) {
          const v4f v = *reinterpret_cast<const v4f*>(b + 16 * (r0 + r) + 4 * q);   // beyond R: unused
#pragma unroll
          for (int c = 0; c < C; ++c) acc[r][c] = v;
        }
      };
    };
    auto zero_init = [&](int, v4f (*acc)[C]) {
#pragma unroll
      for (int r = 0; r < CH; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[r][c] = zero;
    };
    // h = celu(u) in place, t = 2^(u log2(e) / alpha) beside it
    auto celu_chunk = [&](v4f (*acc)[C], v4f (*t)[C]) {
#pragma unroll
      for (int r = 0; r < CH; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            t[r][c][u] = __builtin_amdgcn_exp2f(acc[r][c][u] * inv_alpha_l2);
            acc[r][c][u] = celu_med3(acc[r][c][u], t[r][c][u], alpha);
          }
    };
    // celu'(u) o acc with the FP16 derivatives of the forward pass
    auto times_grad = [&](int r0, v4f (*acc)[C], const uint32_t (*gd)[C][4], int R) {
#pragma unroll
      for (int r = 0; r < CH; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (r0 + r < R) {
              const uint32_t d = gd[(r0 + r) >> 1][c][2 * ((r0 + r) & 1) + (u >> 1)];
              acc[r][c][u] = (u & 1) ? mul_f16<true>(acc[r][c][u], d) : mul_f16<false>(acc[r][c][u], d);
            }
    };
    // ---- layer 1: h1 = celu(W1 x + b1), and celu' for the backward pass
    v8bf h1f[N1 / 32][C];
    uint32_t g1d[N1 / 32][C][4];
    lds_product<N1, K0, Lay::P1, false, CH, C>(W1, xf, lane, bias_init(vb1), [&](int r0, v4f (*acc)[C]) {
      v4f t[CH][C];
      celu_chunk(acc, t);
      chunk_to_frags<N1, CH, C>(r0, acc, h1f);
      chunk_to_grads<N1, CH, C>(r0, t, g1d);
    });
    // ---- layer 2: h2 = celu(W2 h1 + b2), and celu' for the backward pass
    v8bf h2f[N2 / 32][C];
    uint32_t g2d[N2 / 32][C][4];
    lds_product<N2, N1, Lay::P2, false, CH, C>(W2, h1f, lane, bias_init(vb2), [&](int r0, v4f (*acc)[C]) {
      v4f t[CH][C];
      celu_chunk(acc, t);
      chunk_to_frags<N2, CH, C>(r0, acc, h2f);
      chunk_to_grads<N2, CH, C>(r0, t, g2d);
    });
    // ---- layer 3, the output, and delta3 = w4 o celu'(h3)
    v8bf d3f[N3 / 32][C];
    float ep[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ep[c] = 0.f;
    lds_product<N3, N2, Lay::P3, false, CH, C>(W3, h2f, lane, bias_init(vb3), [&](int r0, v4f (*acc)[C]) {
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        if (r0 + r >= N3 / 16) continue;
        const v4f w4 = *reinterpret_cast<const v4f*>(vw4 + 16 * (r0 + r) + 4 * q);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float h = celu_med3(acc[r][c][u], __builtin_amdgcn_exp2f(acc[r][c][u] * inv_alpha_l2), alpha);
            ep[c] = fmaf(w4[u], h, ep[c]);
            acc[r][c][u] = w4[u] * celu_grad_lean(h, inv_alpha);
          }
      }
      chunk_to_frags<N3, CH, C>(r0, acc, d3f);
    });
    // ---- delta2 = (W3^T delta3) o celu'(h2)
    v8bf d2f[N2 / 32][C];
    lds_product<N2, N3, Lay::P3, true, CH, C>(W3, d3f, lane, zero_init, [&](int r0, v4f (*acc)[C]) {
      times_grad(r0, acc, g2d, N2 / 16);
      chunk_to_frags<N2, CH, C>(r0, acc, d2f);
    });
    // ---- delta1 = (W2^T delta2) o celu'(h1)
    v8bf d1f[N1 / 32][C];
    lds_product<N1, N2, Lay::P2, true, CH, C>(W2, d2f, lane, zero_init, [&](int r0, v4f (*acc)[C]) {
      times_grad(r0, acc, g1d, N1 / 16);
      chunk_to_frags<N1, CH, C>(r0, acc, d1f);
    });
    // ---- dE/dx = W1^T delta1, to memory
    lds_product<K0, N1, Lay::P1, true, CH, C>(W1, d1f, lane, zero_init, [&](int r0, v4f (*acc)[C]) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int row = row0 + 16 * c + col;
        if (row < b1_mine) {
#pragma unroll
          for (int r = 0; r < CH; ++r)
            if (r0 + r < K0 / 16)
              *reinterpret_cast<v4f*>(a.g + (int64_t)row * a.stride + 16 * (r0 + r) + 4 * q) = acc[r][c];
        }
      }
    });
    // ---- atomic energies and the tile's FP64 partial sum
    double ev = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float e = ep[c];
      e += __shfl_xor(e, 16, 64);
      e += __shfl_xor(e, 32, 64);
      e += b4;
      const int row = row0 + 16 * c + col;
      if (q == 0 && row < b1_mine) {
        a.e[row] = e;
        ev += (double)e;
      }
    }
    if (a.part != nullptr) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) ev += __shfl_xor(ev, off, 64);
      if (lane == 0) a.part[tiles_before + t] = ev;
    }
  }
}

// One workgroup per CU at most (each holds a species' weights in LDS), no
// more than the tiles need, at least one per species.
template <int K0, int N1, int N2, int N3, int C, int NW>
void launch_lds(const nnp_model& m, const MlpArgs& a, int n, hipStream_t st) {
  const int64_t tiles = (n + 16 * C - 1) / (16 * C) + m.S;
  int64_t G = (tiles + NW - 1) / NW;
  if (G > m.n_cu) G = m.n_cu;
  if (G < m.S) G = m.S;
  hipLaunchKernelGGL((k_mlp_lds<K0, N1, N2, N3, C, NW>), dim3((unsigned)G), dim3(64 * NW), 0, st, a, m.celu_alpha);
}

template <int K0, int N1, int N2, int N3, bool BF16>
hipError_t run_mlp(nnp_model& m, const MlpArgs& a, int n, int variant, hipStream_t st) {
  if (variant == 0) {        // register-resident, one wavefront per 16 atoms
    const int64_t waves = (n + 15) / 16 + m.S;
    hipLaunchKernelGGL((k_mlp_reg<K0, N1, N2, N3, BF16>), dim3((unsigned)((waves * 64 + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, a, m.celu_alpha);
  } else if (variant == 5) {   // 16 atoms per workgroup of eight wavefronts
    const int64_t tiles = (n + 15) / 16 + m.S;
    hipLaunchKernelGGL((k_mlp_split8<K0, N1, N2, N3, BF16, 1, false>), dim3((unsigned)tiles), dim3(512), 0, st, a,
                       m.celu_alpha);
  } else if (variant == 6) {   // eight wavefronts, mixed tiling
    const int64_t tiles = (n + 15) / 16 + m.S;
    hipLaunchKernelGGL((k_mlp_split8<K0, N1, N2, N3, BF16, 2, true>), dim3((unsigned)tiles), dim3(512), 0, st, a,
                       m.celu_alpha);
  } else if (variant == 7) {   // eight wavefronts, 32 atoms per workgroup
    const int64_t tiles = (n + 31) / 32 + m.S;
    hipLaunchKernelGGL((k_mlp_split8<K0, N1, N2, N3, BF16, 2, false>), dim3((unsigned)tiles), dim3(512), 0, st, a,
                       m.celu_alpha);
  } else if (variant == 8 || variant == 9) {   // LDS-resident BF16 weights, a tile per wavefront
    if constexpr (BF16 && K0 <= 128) {
      if (variant == 8)
        launch_lds<K0, N1, N2, N3, 2, 8>(m, a, n, st);    // 32-atom tiles, 2 wavefronts per SIMD
      else
        launch_lds<K0, N1, N2, N3, 1, 16>(m, a, n, st);   // 16-atom tiles, 4 wavefronts per SIMD
    }
  } else if (variant == 4) {   // row split, 32 atoms per workgroup, 16 for the smallest species
    const int64_t tiles = (n + 15) / 16 + m.S;
    hipLaunchKernelGGL((k_mlp_mixed<K0, N1, N2, N3, BF16>), dim3((unsigned)tiles), dim3(256), 0, st, a,
                       m.celu_alpha);
  } else if (variant == 3 && K0 <= 128) {   // row split, 64 atoms per workgroup (narrow networks)
    if constexpr (K0 <= 128) {
      const int64_t tiles = (n + 63) / 64 + m.S;
      hipLaunchKernelGGL((k_mlp_split<K0, N1, N2, N3, BF16, 4>), dim3((unsigned)tiles), dim3(256), 0, st, a,
                         m.celu_alpha);
    }
  } else if (variant >= 2) { // row split, 32 atoms per workgroup
    const int64_t tiles = (n + 31) / 32 + m.S;
    hipLaunchKernelGGL((k_mlp_split<K0, N1, N2, N3, BF16, 2>), dim3((unsigned)tiles), dim3(256), 0, st, a,
                       m.celu_alpha);
  } else {                   // row split, 16 atoms per workgroup
    const int64_t tiles = (n + 15) / 16 + m.S;
    hipLaunchKernelGGL((k_mlp_split<K0, N1, N2, N3, BF16, 1>), dim3((unsigned)tiles), dim3(256), 0, st, a,
                       m.celu_alpha);
  }
  return hipGetLastError();
}

// Networks with the charge output: the same tilings through k_mlp_split_q.
// The register-resident kernel has no charge form; variant 0 runs as 1, and
// the 64-atom tile (narrow networks only) as 2.
template <int K0, int N1, int N2, int N3, bool BF16, int C, bool MIXED, int NW>
void launch_q(const MlpArgs& a, int n, int S, float alpha, hipStream_t st) {
  const int64_t tiles = (C == 2 && !MIXED ? (n + 31) / 32 : (n + 15) / 16) + S;
  hipLaunchKernelGGL((k_mlp_split_q<K0, N1, N2, N3, BF16, C, MIXED, NW>), dim3((unsigned)tiles), dim3(64 * NW), 0,
                     st, a, alpha);
}

template <int K0, int N1, int N2, int N3, bool BF16>
hipError_t run_mlp_q(nnp_model& m, const MlpArgs& a, int n, int variant, hipStream_t st) {
  const float al = m.celu_alpha;
  switch (variant) {
    case 2: case 3: launch_q<K0, N1, N2, N3, BF16, 2, false, 4>(a, n, m.S, al, st); break;
    case 4: launch_q<K0, N1, N2, N3, BF16, 2, true, 4>(a, n, m.S, al, st); break;
    case 5: launch_q<K0, N1, N2, N3, BF16, 1, false, 8>(a, n, m.S, al, st); break;
    case 6: launch_q<K0, N1, N2, N3, BF16, 2, true, 8>(a, n, m.S, al, st); break;
    case 7: launch_q<K0, N1, N2, N3, BF16, 2, false, 8>(a, n, m.S, al, st); break;
    default: launch_q<K0, N1, N2, N3, BF16, 1, false, 4>(a, n, m.S, al, st); break;
  }
  return hipGetLastError();
}

}  // namespace

// Network kernel variant: 0 register-resident (16 atoms per wavefront),
// 1 / 2 / 3 row split over 4 wavefronts with 16 / 32 / 64 atoms per workgroup
// (64 only for the narrow water network; the wide one falls back to 32).  A
// tuned choice for this size wins; otherwise the 32-atom row split, which
// the tuner picked for the water boxes and the H/C/N/O batch in both forms.
int mlp_variant(const nnp_model& m, int n) {
  int v = stage_variant(m, kTuneNetwork, n);
  // the LDS-resident kernels: BF16, the water-sized network, one member
  if ((v == 8 || v == 9) && !(m.prec == NNP_BF16 && m.net_kind == 0 && m.n_members == 1 && m.d_wrow)) v = 2;
  if (v >= 0) return v;
  return 2;
}

hipError_t launch_mlp(nnp_model& m, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  MlpArgs a;
  a.x = m.d_x;
  a.g = m.d_g;
  a.e = m.d_e;
  a.wmat = m.d_wmat;
  a.wvec = m.d_wvec;
  a.bin_start = m.d_bin_start;
  a.n_bins = m.geo.n_bins;
  a.S = m.S;
  a.n_members = m.n_members;
  a.stride = m.stride;
  a.mat_per_species = m.mat_per_species;
  a.vec_per_species = m.vec_per_species;
  a.status = m.d_status;
  a.part = (m.geo.periodic || m.geo.n_bins == 1) ? m.d_part : nullptr;
  a.q = m.charges ? m.d_q : nullptr;
  a.phi_col = m.D;   // the MM potential follows the descriptor
  a.wrow = m.d_wrow;
  a.wrow_per_species = m.wrow_per_species;
  const bool bf = m.prec == NNP_BF16;
  const int v = mlp_variant(m, n);
  m.mlp_cols = v == 3 ? (m.net_kind == 0 ? 4 : 2) : (v == 2 || v == 4 || v == 6 || v == 7 || v == 8 ? 2 : 1);
  m.mlp_mixed = v == 4 || v == 6;
  switch (m.net_kind) {
    case 0:
      return bf ? run_mlp<128, 160, 128, 96, true>(m, a, n, v, st) : run_mlp<128, 160, 128, 96, false>(m, a, n, v, st);
    case 1:
      return bf ? run_mlp<384, 256, 192, 160, true>(m, a, n, v, st) : run_mlp<384, 256, 192, 160, false>(m, a, n, v, st);
    case 2:
      if (m.charges)
        return bf ? run_mlp_q<416, 256, 192, 160, true>(m, a, n, v, st)
                  : run_mlp_q<416, 256, 192, 160, false>(m, a, n, v, st);
      return bf ? run_mlp<416, 256, 192, 160, true>(m, a, n, v, st) : run_mlp<416, 256, 192, 160, false>(m, a, n, v, st);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace nnp
