// Host-side weight handling: the seeded draw (SplitMix64 + Box-Muller) and the
// packing of every matrix into MFMA fragment order.
#include <cmath>
#include <cstring>

#include "nnp_internal.h"

namespace nnp {
namespace {

// SplitMix64 output `counter` (0-based) of the stream started at `seed`
// (Steele, Lea & Flood, "Fast splittable pseudorandom number generators", 2014).
inline uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline double uniform01(uint64_t seed, uint64_t counter) {
  return (double)(splitmix64(seed, counter) >> 11) * 0x1.0p-53;
}

// Standard normal t of the stream: Box-Muller on uniforms 2t and 2t+1.
inline double normal(uint64_t seed, uint64_t start, uint64_t t) {
  double u0 = uniform01(seed, start + 2 * t);
  double u1 = uniform01(seed, start + 2 * t + 1);
  return std::sqrt(-2.0 * std::log(1.0 - u0)) * std::cos(2.0 * M_PI * u1);
}

inline uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Pack M [R x C] (row-major, leading dimension ld, zero outside rows x cols)
// as A-operand fragments.  FP32 (16x16x4): element (rt, kb, lane, s) =
// M[16 rt + lane%16][16 kb + 4 (lane/16) + s].  BF16 (16x16x32): element
// (rt, kb, lane, j) = M[16 rt + lane%16][32 kb + k(j)], k(j) = 4 (lane/16) + j
// for j < 4 and 16 + 4 (lane/16) + (j - 4) otherwise -- the same K permutation
// the kernel applies to the activations.
template <typename Get>
void pack_matrix(Get get, int R, int C, bool bf16, std::vector<uint8_t>& out) {
  if (!bf16) {
    size_t base = out.size();
    out.resize(base + (size_t)R * C * 4);
    float* d = reinterpret_cast<float*>(out.data() + base);
    for (int rt = 0; rt < R / 16; ++rt)
      for (int kb = 0; kb < C / 16; ++kb)
        for (int lane = 0; lane < 64; ++lane)
          for (int s = 0; s < 4; ++s)
            d[(((size_t)rt * (C / 16) + kb) * 64 + lane) * 4 + s] =
                get(16 * rt + (lane & 15), 16 * kb + 4 * (lane >> 4) + s);
  } else {
    size_t base = out.size();
    out.resize(base + (size_t)R * C * 2);
    uint16_t* d = reinterpret_cast<uint16_t*>(out.data() + base);
    for (int rt = 0; rt < R / 16; ++rt)
      for (int kb = 0; kb < C / 32; ++kb)
        for (int lane = 0; lane < 64; ++lane)
          for (int j = 0; j < 8; ++j) {
            int q = lane >> 4;
            int k = 32 * kb + (j < 4 ? 4 * q + j : 16 + 4 * q + (j - 4));
            d[(((size_t)rt * (C / 32) + kb) * 64 + lane) * 8 + j] = bf16_rne(get(16 * rt + (lane & 15), k));
          }
  }
}

}  // namespace

void draw_weights(uint64_t seed, const std::vector<int>& widths, int n_species, int n_members,
                  std::vector<float>& out) {
  out.clear();
  uint64_t counter = 0;
  for (int m = 0; m < n_members; ++m)
    for (int s = 0; s < n_species; ++s)
      for (size_t l = 0; l + 1 < widths.size(); ++l) {
        int fi = widths[l], fo = widths[l + 1];
        double std_w = std::sqrt(2.0 / (double)(fi + fo));
        uint64_t nw = (uint64_t)fi * fo;
        for (uint64_t t = 0; t < nw; ++t) out.push_back((float)(normal(seed, counter, t) * std_w));
        counter += 2 * nw;
        for (int t = 0; t < fo; ++t) out.push_back((float)(normal(seed, counter, (uint64_t)t) * 0.1));
        counter += 2 * (uint64_t)fo;
      }
}

void pack_weights(const nnp_model& m, std::vector<uint8_t>& mat, std::vector<float>& vec,
                  int64_t& mat_per_species, int64_t& vec_per_species) {
  const bool bf = m.prec == NNP_BF16;
  const int K0 = m.widths[0];          // real input width
  const int K0p = m.stride;            // padded
  const int N1 = m.widths[1], N2 = m.widths[2], N3 = m.widths[3];
  mat.clear();
  vec.clear();
  size_t off = 0;
  int64_t mat_elems = (int64_t)N1 * K0p + (int64_t)N2 * N1 + (int64_t)N3 * N2 + (int64_t)K0p * N1 +
                      (int64_t)N1 * N2 + (int64_t)N2 * N3;
  mat_per_species = mat_elems;
  const int n_out = m.charges ? 2 : 1;   // energy, and the predicted charge
  vec_per_species = N1 + N2 + N3 + n_out * (N3 + 4);
  for (int mem = 0; mem < m.n_members; ++mem)
    for (int s = 0; s < m.S; ++s) {
      const float* W1 = m.w_host.data() + off;
      const float* b1 = W1 + (size_t)N1 * K0;
      const float* W2 = b1 + N1;
      const float* b2 = W2 + (size_t)N2 * N1;
      const float* W3 = b2 + N2;
      const float* b3 = W3 + (size_t)N3 * N2;
      const float* W4 = b3 + N3;                 // [n_out x N3]
      const float* b4 = W4 + (size_t)n_out * N3;  // [n_out]
      off = (size_t)(b4 + n_out - m.w_host.data());
      auto g1 = [&](int r, int c) { return c < K0 ? W1[(size_t)r * K0 + c] : 0.f; };
      auto g2 = [&](int r, int c) { return W2[(size_t)r * N1 + c]; };
      auto g3 = [&](int r, int c) { return W3[(size_t)r * N2 + c]; };
      auto t1 = [&](int r, int c) { return r < K0 ? W1[(size_t)c * K0 + r] : 0.f; };
      auto t2 = [&](int r, int c) { return W2[(size_t)c * N1 + r]; };
      auto t3 = [&](int r, int c) { return W3[(size_t)c * N2 + r]; };
      pack_matrix(g1, N1, K0p, bf, mat);
      pack_matrix(g2, N2, N1, bf, mat);
      pack_matrix(g3, N3, N2, bf, mat);
      pack_matrix(t1, K0p, N1, bf, mat);
      pack_matrix(t2, N1, N2, bf, mat);
      pack_matrix(t3, N2, N3, bf, mat);
      vec.insert(vec.end(), b1, b1 + N1);
      vec.insert(vec.end(), b2, b2 + N2);
      vec.insert(vec.end(), b3, b3 + N3);
      for (int o = 0; o < n_out; ++o) {   // output row o: weights, bias, 3 zeros of padding
        vec.insert(vec.end(), W4 + (size_t)o * N3, W4 + (size_t)(o + 1) * N3);
        vec.push_back(b4[o]);
        vec.push_back(0.f);
        vec.push_back(0.f);
        vec.push_back(0.f);
      }
    }
}

void pack_rows_bf16(const nnp_model& m, std::vector<uint16_t>& out, int64_t& per_species) {
  const int K0 = m.widths[0], K0p = m.stride;
  const int N1 = m.widths[1], N2 = m.widths[2], N3 = m.widths[3];
  const int n_out = m.charges ? 2 : 1;
  per_species = (int64_t)N1 * K0p + (int64_t)N2 * N1 + (int64_t)N3 * N2;
  out.clear();
  size_t off = 0;
  for (int mem = 0; mem < m.n_members; ++mem)
    for (int s = 0; s < m.S; ++s) {
      const float* W1 = m.w_host.data() + off;
      const float* W2 = W1 + (size_t)N1 * K0 + N1;
      const float* W3 = W2 + (size_t)N2 * N1 + N2;
      off = (size_t)(W3 + (size_t)N3 * N2 + N3 + (size_t)n_out * N3 + n_out - m.w_host.data());
      for (int r = 0; r < N1; ++r)
        for (int c = 0; c < K0p; ++c) out.push_back(c < K0 ? bf16_rne(W1[(size_t)r * K0 + c]) : 0);
      for (int r = 0; r < N2; ++r)
        for (int c = 0; c < N1; ++c) out.push_back(bf16_rne(W2[(size_t)r * N1 + c]));
      for (int r = 0; r < N3; ++r)
        for (int c = 0; c < N2; ++c) out.push_back(bf16_rne(W3[(size_t)r * N2 + c]));
    }
}

}  // namespace nnp
