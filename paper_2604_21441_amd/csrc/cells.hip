// Cell-list neighbour search over the atoms of the index group (Methods: the
// interface's ML subsystem): binning, a stable counting sort by
// key = species * n_bins + bin, and per-atom neighbour lists grouped by
// species; also the lists built from a caller's pair list.  A bin is a cell of the periodic box, or a whole system in batched
// mode (open systems small enough for an all-pairs scan per system).
//
// The binning and the distance predicate are integer-exact functions of the
// FP32 inputs: every operation below is a single IEEE FP32 operation in a
// fixed order with floating-point contraction disabled, so an FP32 reference
// that performs the same operations reproduces the bins, the permutation and
// the neighbour sets bit for bit.
#include <algorithm>

#include <cmath>

#include "nnp_internal.h"

namespace nnp {
namespace {

constexpr int kBlock = 256;

// Position of NNP-local atom t: a system atom, or a link atom placed on its
// cut bond (eq. 4; bond vector under the minimum image when periodic).
__device__ __forceinline__ float3 nnp_position(const float* __restrict__ pos, int a, const LinkArgs& L,
                                               const Geometry& g) {
  if (a >= 0) return make_float3(pos[3 * (int64_t)a], pos[3 * (int64_t)a + 1], pos[3 * (int64_t)a + 2]);
  const int l = -1 - a;
  const int ml = L.ml[l], mm = L.mm[l];
  float3 p = make_float3(pos[3 * (int64_t)ml], pos[3 * (int64_t)ml + 1], pos[3 * (int64_t)ml + 2]);
  float ux = pos[3 * (int64_t)mm] - p.x, uy = pos[3 * (int64_t)mm + 1] - p.y, uz = pos[3 * (int64_t)mm + 2] - p.z;
  if (g.periodic) {
    ux -= g.box[0] * rintf(ux * g.inv_box[0]);
    uy -= g.box[1] * rintf(uy * g.inv_box[1]);
    uz -= g.box[2] * rintf(uz * g.inv_box[2]);
  }
  const float s = L.d / sqrtf(ux * ux + uy * uy + uz * uz);
  return make_float3(p.x + s * ux, p.y + s * uy, p.z + s * uz);
}

// Bin of one position in the periodic grid.
__device__ __forceinline__ int cell_of(float x, float y, float z, const Geometry& g) {
#pragma clang fp contract(off)
  float c[3] = {x, y, z};
  int ci[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float t = c[k] * g.inv_box[k];
    float f = floorf(t);
    float fl = f * g.box[k];
    float w = c[k] - fl;
    float sc = w * g.cell_scale[k];
    int q = (int)floorf(sc);
    q = q < 0 ? 0 : q;
    q = q > g.nc[k] - 1 ? g.nc[k] - 1 : q;
    ci[k] = q;
  }
  return (ci[0] * g.nc[1] + ci[1]) * g.nc[2] + ci[2];
}

__global__ __launch_bounds__(kBlock) void k_stage(const float* __restrict__ pos, int n,
                                                  const int* __restrict__ idx,
                                                  const int* __restrict__ sigma,
                                                  const int* __restrict__ sys, Geometry g, LinkArgs L,
                                                  int* __restrict__ key, int* __restrict__ rank,
                                                  float4* __restrict__ stg,
                                                  int* __restrict__ bin_count, int* __restrict__ status) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float3 p = nnp_position(pos, idx[t], L, g);
  float x = p.x, y = p.y, z = p.z;
  if (g.periodic) stg[t] = make_float4(x, y, z, __int_as_float(sigma[t]));   // for the bin sort
  int bin;
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    atomicOr(status, kStatusNonFinite);
    bin = g.periodic ? 0 : sys[t];
  } else {
    bin = g.periodic ? cell_of(x, y, z, g) : sys[t];
  }
  int k = sigma[t] * g.n_bins + bin;
  key[t] = k;
  if (g.periodic) {
    rank[t] = atomicAdd(&bin_count[k], 1);   // arrival order among the atoms of the key
    return;
  }
  // Open systems (bins are systems): a system's atoms are contiguous, so a
  // wavefront holds few distinct keys and per-atom atomics would queue on the
  // same few counters.  One atomic per distinct key and wavefront instead (the
  // system ranking places the atoms itself; no arrival rank is needed).
  const int lane = threadIdx.x & 63;
  uint64_t todo = __builtin_amdgcn_ballot_w64(true);
  while (todo != 0) {
    const int leader = __builtin_ctzll(todo);
    const int lk = __builtin_amdgcn_readlane(k, leader);
    const uint64_t same = __builtin_amdgcn_ballot_w64(k == lk);
    if (lane == leader) atomicAdd(&bin_count[lk], (int)__popcll(same));
    todo &= ~same;
  }
}

// Exclusive scans of the bin histogram by one workgroup.
//   start: species-major order (key = species * n_bins + bin), the slot
//     order of the sorted arrays;
//   cmstart[bin * S + species]: bin-major order, the order in which the
//     per-atom kernels visit the slots (all species of a cell or system
//     together, so neighbouring atoms are processed close in time).
// Chunks of kScanThreads * PER entries are staged through LDS so that every global
// load and store is coalesced (per-thread runs of consecutive entries read
// straight from memory are several times slower); each thread scans
// PER consecutive entries of the staged chunk, PER being the smallest power
// of two for which one chunk holds the whole histogram (at most 16; larger
// histograms go to the many-workgroup scan, k_scan_part and k_scan_fin).  Sizing the chunk to the histogram
// matters: one workgroup does all of this work, and with 16 entries per
// thread a 1,024-bin scan took 6.8 us.  The histogram itself is left as it
// is (the bin sort clears it).
constexpr int kScanThreads = 1024;
constexpr int kScanPerMax = 16;
constexpr int kScanChunk = kScanThreads * kScanPerMax;   // largest chunk

// LDS index of chunk entry i: one pad word after every PER entries, so the
// per-thread runs start in different banks (stride PER + 1 is odd).
template <int PER>
__device__ __forceinline__ int scan_pad(int i) { return PER == 1 ? i : i + i / PER; }
template <int PER>
constexpr int scan_lds_words() { return PER == 1 ? kScanThreads : kScanThreads * (PER + 1); }

// Exclusive prefix of v over the workgroup (thread order); *total receives the sum.
__device__ __forceinline__ int block_exclusive(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(inc, off, 64);
    if (lane >= off) inc += u;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    const int w = lane < kScanThreads / 64 ? wsum[lane] : 0;
    int wi = w;
#pragma unroll
    for (int off = 1; off < kScanThreads / 64; off <<= 1) {
      const int u = __shfl_up(wi, off, 64);
      if (lane >= off) wi += u;
    }
    if (lane < kScanThreads / 64) wsum[kScanThreads / 64 + lane] = wi - w;
    if (lane == kScanThreads / 64 - 1) wsum[2 * (kScanThreads / 64)] = wi;
  }
  __syncthreads();
  const int ex = wsum[kScanThreads / 64 + wave] + inc - v;
  *total = wsum[2 * (kScanThreads / 64)];
  __syncthreads();   // wsum is reused by the next call
  return ex;
}

// Scan of the staged chunk buf[0 .. kScanThreads * PER) in place (exclusive, plus carry).
template <int PER>
__device__ __forceinline__ void scan_chunk(int* buf, int* wsum, int* carry) {
  int v[PER];
  int sum = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    v[u] = buf[scan_pad<PER>(threadIdx.x * PER + u)];
    sum += v[u];
  }
  int total;
  int run = block_exclusive(sum, wsum, &total) + *carry;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    buf[scan_pad<PER>(threadIdx.x * PER + u)] = run;
    run += v[u];
  }
  *carry += total;
  __syncthreads();
}

template <int PER>
__global__ __launch_bounds__(kScanThreads) void k_scan(const int* __restrict__ count, int* __restrict__ start,
                                                       int* __restrict__ cmstart, int S, int n_bins) {
  __shared__ int wsum[2 * (kScanThreads / 64) + 1];
  __shared__ int buf[scan_lds_words<PER>()];
  __shared__ int bufc[scan_lds_words<PER>()];
  const int nb = S * n_bins;
  int carry = 0;
  if (nb <= kScanThreads * PER) {
    // one chunk: the histogram is read once and both scans run from LDS
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = u * kScanThreads + threadIdx.x;
      bufc[scan_pad<PER>(i)] = i < nb ? count[i] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int b = u * kScanThreads + threadIdx.x;
      int t = 0;
#pragma unroll
      for (int s = 0; s < kMaxSpecies; ++s)
        if (s < S && b < n_bins) t += bufc[scan_pad<PER>(s * n_bins + b)];
      buf[scan_pad<PER>(b)] = t;
    }
    __syncthreads();
    scan_chunk<PER>(buf, wsum, &carry);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int b = u * kScanThreads + threadIdx.x;
      if (b < n_bins) {
        int r = buf[scan_pad<PER>(b)];
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s)
          if (s < S) {
            cmstart[b * S + s] = r;
            r += bufc[scan_pad<PER>(s * n_bins + b)];
          }
      }
    }
    __syncthreads();
    carry = 0;
    scan_chunk<PER>(bufc, wsum, &carry);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = u * kScanThreads + threadIdx.x;
      if (i < nb) start[i] = bufc[scan_pad<PER>(i)];
    }
    if (threadIdx.x == 0) start[nb] = carry;
  }
}

// Histograms beyond one chunk: the same two scans over many workgroups, in
// two launches.  Workgroup w < ca takes species-major chunk w (counts), the
// others bin-major chunk w - ca (per-bin totals over the species); each chunk
// holds kScanPartChunk = kScanThreads * 4 entries.  k_scan_part writes the
// chunk totals, k_scan_fin scans each chunk again starting from the sum of
// the earlier chunks of its order.  One workgroup scanning 35,152 bins took
// 38 us.
constexpr int kScanPartPer = kScanPartChunk / kScanThreads;
static_assert(kScanPartPer * kScanThreads == kScanPartChunk, "whole entries per thread");

__device__ __forceinline__ int scan_entry(const int* __restrict__ count, bool bin_major, int e, int S, int n_bins) {
  if (!bin_major) return count[e];
  int t = 0;
#pragma unroll
  for (int s = 0; s < kMaxSpecies; ++s)
    if (s < S) t += count[s * n_bins + e];
  return t;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_part(const int* __restrict__ count, int S, int n_bins,
                                                            int ca, int* __restrict__ part) {
  __shared__ int wsum[2 * (kScanThreads / 64) + 1];
  const bool bin_major = (int)blockIdx.x >= ca;
  const int c = bin_major ? (int)blockIdx.x - ca : (int)blockIdx.x;
  const int len = bin_major ? n_bins : S * n_bins;
  int sum = 0;
#pragma unroll
  for (int u = 0; u < kScanPartPer; ++u) {
    const int e = c * kScanPartChunk + u * kScanThreads + threadIdx.x;
    if (e < len) sum += scan_entry(count, bin_major, e, S, n_bins);
  }
  int total;
  block_exclusive(sum, wsum, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_fin(const int* __restrict__ count, int* __restrict__ start,
                                                           int* __restrict__ cmstart, int S, int n_bins, int ca,
                                                           const int* __restrict__ part) {
  __shared__ int wsum[2 * (kScanThreads / 64) + 1];
  __shared__ int buf[scan_lds_words<kScanPartPer>()];
  __shared__ int s_carry;
  const bool bin_major = (int)blockIdx.x >= ca;
  const int c = bin_major ? (int)blockIdx.x - ca : (int)blockIdx.x;
  const int first = bin_major ? ca : 0;
  const int nb = S * n_bins, len = bin_major ? n_bins : nb;
  if (threadIdx.x < 64) {   // the earlier chunks of this order
    int v = 0;
    for (int k = first + (int)threadIdx.x; k < (int)blockIdx.x; k += 64) v += part[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x == 0) s_carry = v;
  }
  const int c0 = c * kScanPartChunk;
#pragma unroll
  for (int u = 0; u < kScanPartPer; ++u) {
    const int i = u * kScanThreads + threadIdx.x;
    buf[scan_pad<kScanPartPer>(i)] = c0 + i < len ? scan_entry(count, bin_major, c0 + i, S, n_bins) : 0;
  }
  __syncthreads();
  int carry = s_carry;
  scan_chunk<kScanPartPer>(buf, wsum, &carry);
#pragma unroll
  for (int u = 0; u < kScanPartPer; ++u) {
    const int i = u * kScanThreads + threadIdx.x, e = c0 + i;
    if (e < len) {
      int r = buf[scan_pad<kScanPartPer>(i)];
      if (bin_major) {
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s)
          if (s < S) {
            cmstart[e * S + s] = r;
            r += count[s * n_bins + e];
          }
      } else {
        start[e] = r;
      }
    }
  }
  if (!bin_major && c0 + kScanPartChunk >= len && threadIdx.x == 0) start[nb] = carry;
}

// Provisional slots: start of the key plus the atom's arrival rank.
__global__ __launch_bounds__(kBlock) void k_scatter(const int* __restrict__ key, const int* __restrict__ rank, int n,
                                                    const int* __restrict__ start, int* __restrict__ tmp) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  tmp[start[key[t]] + rank[t]] = t;
}

// Scan and scatter in one launch, for histograms of at most one chunk: every
// workgroup stages the histogram in LDS and scans it itself (a few KB to a
// few tens of KB from L2, cheaper than a kernel boundary); workgroup 0 also
// writes both scans for the later kernels.  Then each thread places one
// atom at start[key] + rank.
template <int PER>
__global__ __launch_bounds__(kScanThreads) void k_scan_scatter(const int* __restrict__ count, int* __restrict__ start,
                                                               int* __restrict__ cmstart, int S, int n_bins,
                                                               const int* __restrict__ key,
                                                               const int* __restrict__ rank, int n,
                                                               int* __restrict__ tmp) {
  __shared__ int wsum[2 * (kScanThreads / 64) + 1];
  __shared__ int buf[scan_lds_words<PER>()];
  __shared__ int bufc[scan_lds_words<PER>()];
  const int nb = S * n_bins;   // <= kScanThreads * PER (checked by the launcher)
  const int t = blockIdx.x * kScanThreads + threadIdx.x;
  const int k = t < n ? key[t] : 0;
  const int rk = t < n ? rank[t] : 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = u * kScanThreads + threadIdx.x;
    bufc[scan_pad<PER>(i)] = i < nb ? count[i] : 0;
  }
  __syncthreads();
  int carry = 0;
  if (blockIdx.x == 0) {   // bin-major starts (workgroup-uniform branch)
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int b = u * kScanThreads + threadIdx.x;
      int tot = 0;
#pragma unroll
      for (int s = 0; s < kMaxSpecies; ++s)
        if (s < S && b < n_bins) tot += bufc[scan_pad<PER>(s * n_bins + b)];
      buf[scan_pad<PER>(b)] = tot;
    }
    __syncthreads();
    scan_chunk<PER>(buf, wsum, &carry);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int b = u * kScanThreads + threadIdx.x;
      if (b < n_bins) {
        int r = buf[scan_pad<PER>(b)];
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s)
          if (s < S) {
            cmstart[b * S + s] = r;
            r += bufc[scan_pad<PER>(s * n_bins + b)];
          }
      }
    }
    __syncthreads();
    carry = 0;
  }
  scan_chunk<PER>(bufc, wsum, &carry);   // species-major starts, in place
  if (blockIdx.x == 0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = u * kScanThreads + threadIdx.x;
      if (i < nb) start[i] = bufc[scan_pad<PER>(i)];
    }
    if (threadIdx.x == 0) start[nb] = carry;
  }
  if (t < n) tmp[bufc[scan_pad<PER>(k)] + rk] = t;
}

// Small periodic systems: the whole cell list in one workgroup, through LDS.
// LDS histogram atomics give arrival ranks, both scans run in LDS, and each
// thread then places its own atoms: the stable slot of atom t is the start of
// its key plus the number of atoms of that key with a smaller index, counted
// in the key's segment of the arrival-order scatter.  One launch instead of
// three (binning, scan + scatter, bin sort), with the same outputs bit for
// bit.  The device histogram is not touched (it stays zero).
constexpr int kSmallCells = 2048;   // atoms; LDS: 2 padded scan buffers + 2 ints per atom
static_assert(kSmallCells % kScanThreads == 0, "whole atoms per thread");

template <int PER>
__global__ __launch_bounds__(kScanThreads) void k_cells_small(const float* __restrict__ pos, int n,
                                                              const int* __restrict__ idx,
                                                              const int* __restrict__ sigma, Geometry g,
                                                              LinkArgs L, int S, int* __restrict__ key,
                                                              int* __restrict__ bin_start,
                                                              int* __restrict__ perm, float4* __restrict__ spos,
                                                              int* __restrict__ slot_atom,
                                                              int* __restrict__ order, int* __restrict__ sbin,
                                                              int* __restrict__ islot, int* __restrict__ pcount,
                                                              int* __restrict__ status) {
  __shared__ int wsum[2 * (kScanThreads / 64) + 1];
  __shared__ int hist[scan_lds_words<PER>()];   // counts per key, then species-major starts
  __shared__ int bmaj[scan_lds_words<PER>()];   // totals per bin, then bin-major starts
  __shared__ int tmp[kSmallCells];               // atoms of each key in arrival order
  __shared__ int kr[kSmallCells];                // key | arrival rank << 15
  const int nb = S * g.n_bins;                   // <= kScanThreads * PER <= 2^14 (checked by the launcher)
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < PER; ++u) hist[scan_pad<PER>(u * kScanThreads + tid)] = 0;
  __syncthreads();
  // each thread owns atoms tid + u * kScanThreads and keeps their data in registers
  constexpr int kOwn = kSmallCells / kScanThreads;
  float3 pp[kOwn];
  int aa[kOwn], ss[kOwn];
#pragma unroll
  for (int u = 0; u < kOwn; ++u) {
    const int t = u * kScanThreads + tid;
    if (t >= n) continue;
    aa[u] = idx[t];
    ss[u] = sigma[t];
    pp[u] = nnp_position(pos, aa[u], L, g);
    int bin = 0;
    if (!(isfinite(pp[u].x) && isfinite(pp[u].y) && isfinite(pp[u].z)))
      atomicOr(status, kStatusNonFinite);
    else
      bin = cell_of(pp[u].x, pp[u].y, pp[u].z, g);
    const int k = ss[u] * g.n_bins + bin;
    key[t] = k;
    const int r = atomicAdd(&hist[scan_pad<PER>(k)], 1);
    kr[t] = k | (r << 15);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int b = u * kScanThreads + tid;
    int tot = 0;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s)
      if (s < S && b < g.n_bins) tot += hist[scan_pad<PER>(s * g.n_bins + b)];
    bmaj[scan_pad<PER>(b)] = tot;
  }
  __syncthreads();
  int carry = 0;
  scan_chunk<PER>(bmaj, wsum, &carry);
  carry = 0;
  scan_chunk<PER>(hist, wsum, &carry);
  auto start_of = [&](int k) { return k < nb ? hist[scan_pad<PER>(k)] : n; };
  for (int i = tid; i <= nb; i += kScanThreads) bin_start[i] = start_of(i);
  for (int t = tid; t < n; t += kScanThreads) {
    const int v = kr[t];
    tmp[start_of(v & 0x7fff) + (v >> 15)] = t;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kOwn; ++u) {
    const int t = u * kScanThreads + tid;
    if (t >= n) continue;
    const int k = kr[t] & 0x7fff;
    const int b0 = start_of(k), b1 = start_of(k + 1);
    int rank = 0;
    for (int e = b0; e < b1; ++e) rank += tmp[e] < t;
    const int slot = b0 + rank;
    const int sp = k / g.n_bins, bin = k - sp * g.n_bins;
    int o0 = bmaj[scan_pad<PER>(bin)];   // bin-major: earlier bins, then earlier species of this bin
    for (int s = 0; s < sp; ++s) o0 += start_of(s * g.n_bins + bin + 1) - start_of(s * g.n_bins + bin);
    const int cz = bin % g.nc[2], cxy = bin / g.nc[2];
    perm[slot] = t;
    order[o0 + rank] = slot;
    sbin[slot] = ((cxy / g.nc[1]) << 20) | ((cxy % g.nc[1]) << 10) | cz;
    islot[t] = slot;
    pcount[slot] = 0;
    spos[slot] = make_float4(pp[u].x, pp[u].y, pp[u].z, __int_as_float(ss[u]));
    slot_atom[slot] = aa[u];
  }
}

// One wavefront per bin: the atomically scattered entries of the bin are
// ranked by atom index (a stable order independent of the atomic order), and
// the sorted positions / species / atom indices are written per slot, and
// each slot's place in the bin-major visiting order.
__global__ __launch_bounds__(kBlock) void k_binsort(const int* __restrict__ start, int n_bins_total,
                                                    const int* __restrict__ tmp,
                                                    const float4* __restrict__ stg,
                                                    const int* __restrict__ idx, Geometry g,
                                                    const int* __restrict__ cmstart, int S,
                                                    int* __restrict__ perm,
                                                    float4* __restrict__ spos,
                                                    int* __restrict__ slot_atom,
                                                    int* __restrict__ order, int* __restrict__ sbin,
                                                    int* __restrict__ islot, int* __restrict__ pcount,
                                                    int* __restrict__ count) {
  int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (wave >= n_bins_total) return;
  if (lane == 0) count[wave] = 0;   // the histogram starts from zero in the next call
  int b0 = start[wave], b1 = start[wave + 1];
  const int sp = wave / g.n_bins, bin = wave - sp * g.n_bins;
  const int o0 = cmstart[bin * S + sp];
  // the cell's coordinates, packed for the neighbour search
  const int cz = bin % g.nc[2], cxy = bin / g.nc[2];
  const int packed = ((cxy / g.nc[1]) << 20) | ((cxy % g.nc[1]) << 10) | cz;
  const int cnt = b1 - b0;
  // bins of up to 64 atoms: one entry per lane, ranked against the others
  // with lane reads (no memory round trip per comparison)
  const int mine = lane < cnt ? tmp[b0 + lane] : 0;
  for (int e = b0 + lane; e < b1; e += 64) {
    int t = tmp[e];
    int rank = 0;
    if (cnt <= 64) {
      for (int q = 0; q < cnt; ++q) rank += __builtin_amdgcn_readlane(mine, q) < t;
    } else {
      for (int q = b0; q < b1; ++q) rank += tmp[q] < t;
    }
    int slot = b0 + rank;
    perm[slot] = t;
    order[o0 + rank] = slot;
    sbin[slot] = packed;
    islot[t] = slot;
    pcount[slot] = 0;
    spos[slot] = stg[t];   // staged by k_stage: no second trip through idx and pos
    slot_atom[slot] = idx[t];
  }
}

// Open systems (one bin per system): the stable slot of every atom is found
// directly, one wavefront per system.  The system's atoms are taken in input
// order, 64 at a time; for each species a ballot gives every atom its rank
// among the earlier atoms of its species, so slot = bin start + rank.  No
// atomics and no in-bin sort are needed, whatever the system size.
__global__ __launch_bounds__(64) void k_rank_systems(const int* __restrict__ sys_off, int n_sys, int S,
                                                      const int* __restrict__ bin_start,
                                                      const int* __restrict__ sigma,
                                                      const int* __restrict__ idx, const float* __restrict__ pos,
                                                      Geometry g, LinkArgs L, const int* __restrict__ cmstart,
                                                      int* __restrict__ perm, float4* __restrict__ spos,
                                                      int* __restrict__ slot_atom, int* __restrict__ order,
                                                      int* __restrict__ count, int* __restrict__ sbin,
                                                      int* __restrict__ islot, int* __restrict__ pcount) {
  const int m = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane < S) count[lane * n_sys + m] = 0;   // the histogram starts from zero in the next call
  const int t0 = sys_off[m], t1 = sys_off[m + 1];
  const uint64_t lt = __lanemask_lt();
  int base[kMaxSpecies] = {0, 0, 0, 0}, first[kMaxSpecies], cm[kMaxSpecies];
#pragma unroll
  for (int s = 0; s < kMaxSpecies; ++s) {   // per-system constants (wave-uniform)
    first[s] = s < S ? bin_start[s * n_sys + m] : 0;
    cm[s] = s < S ? cmstart[m * S + s] : 0;
  }
  // the next block of 64 atoms is loaded while the current one is placed
  auto fetch = [&](int t, int& sg, int& a) {
    sg = -1;
    a = 0;
    if (t < t1) {
      sg = sigma[t];
      a = idx[t];
    }
  };
  int sg_n, a_n;
  fetch(t0 + lane, sg_n, a_n);
  for (int c0 = t0; c0 < t1; c0 += 64) {
    const int t = c0 + lane;
    const bool ok = t < t1;
    const int sg = sg_n, a = a_n;
    const float3 p = ok ? nnp_position(pos, a, L, g) : make_float3(0.f, 0.f, 0.f);
    if (c0 + 64 < t1) fetch(t + 64, sg_n, a_n);
    int slot = 0, rank = 0, o = 0;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      if (s < S) {
        const uint64_t mk = __ballot(sg == s);
        if (sg == s) {
          rank = base[s] + __popcll(mk & lt);
          slot = first[s] + rank;
          o = cm[s] + rank;
        }
        base[s] += __popcll(mk);
      }
    }
    if (ok) {
      perm[slot] = t;
      order[o] = slot;
      sbin[slot] = m;
      islot[t] = slot;
      pcount[slot] = 0;
      spos[slot] = make_float4(p.x, p.y, p.z, __int_as_float(sg));
      slot_atom[slot] = a;
    }
  }
}

struct NeighArgs {
  const int* order;        // bin-major visiting order of the slots
  const int* sbin;         // packed cell coordinates (periodic) or system of each slot
  const float4* spos;
  const int* perm;
  const int* key;
  const int* bin_start;
  int n, S;
  float rc2, rca2;
  float cull2;             // (sqrt(rc2) + kCullMargin)^2: stencil cells beyond it hold no neighbour
  int* rad;
  int* ang;
  int* angpos;
  int* rad_off;
  int* ang_off;
  int max_rad, max_ang;
  int* status;
};

constexpr int kMaxStencil = 27;

// One wavefront per sorted slot i.  For each species, the candidate atoms of
// the (deduplicated) 27-cell stencil are visited in ascending cell order --
// hence ascending slot order -- one candidate per lane, and the accepted ones
// are compacted with a ballot, so every species segment of a list is sorted
// by slot.  Angular neighbours (r < rc_ang) also record their position in
// the radial list.  Lists never hold more than their capacity; an overflow
// sets the device status word.
// Candidates of one species per atom held in LDS (flattened stencil ranges);
// a longer candidate sequence falls back to a binary search over the ranges.
constexpr int kCandCap = 1024;
// Distance (A) added to the cutoff before a stencil cell is skipped.  Cell
// assignment and the distance test round positions to a few FP32 ulps,
// about 1e-3 A for coordinates of 10^4 A, so skipping is exact for inputs
// within many box lengths of the origin.
constexpr float kCullMargin = 0.02f;

__global__ __launch_bounds__(64) void k_neighbours(NeighArgs a, Geometry g) {
#pragma clang fp contract(off)
  __shared__ int s_start[kMaxStencil];
  __shared__ int s_off[kMaxStencil + 1];
  __shared__ int s_cand[kCandCap];
  const int i = a.order[xcd_block(blockIdx.x, gridDim.x)];
  const int lane = threadIdx.x;
  const float4 pi = a.spos[i];
  const int sb = a.sbin[i];
  const MinImage mi = min_image_at(g, i);
  // Stencil cells in ascending id order: per dimension the (wrapped)
  // coordinates {c-1, c, c+1} are sorted, and ids are lexicographic in
  // (x, y, z).  Lane l < nst takes the l-th of them.
  int nst = 1;
  int my_cell = sb;   // open systems: the system's bin
  bool culled = false;
  if (g.periodic) {
    const int c[3] = {sb >> 20, (sb >> 10) & 1023, sb & 1023};
    int nd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) nd[k] = g.nc[k] >= 3 ? 3 : g.nc[k];
    nst = nd[0] * nd[1] * nd[2];
    const int l = lane < nst ? lane : 0;
    int o[3];
    if (nst == 27) {
      o[0] = l / 9; o[1] = (l / 3) % 3; o[2] = l % 3;
    } else {
      o[0] = l / (nd[1] * nd[2]); o[1] = (l / nd[2]) % nd[1]; o[2] = l % nd[2];
    }
    // A stencil cell whose nearest point lies beyond the cutoff (plus
    // kCullMargin) holds no neighbour of this centre: its lane offers no
    // candidates.  The gap per dimension is the centre's offset inside its
    // own cell (lower neighbour) or the rest of the cell (upper neighbour).
    const float pc[3] = {pi.x, pi.y, pi.z};
    float gap2 = 0.f;
    int v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int n = g.nc[k];
      if (n < 3) {   // every cell of the dimension is in the stencil
        v[k] = o[k];
        continue;
      }
      // offset of the o-th sorted coordinate: c = 0 gives {0, 1, n-1},
      // c = n-1 gives {0, n-2, n-1}, otherwise {c-1, c, c+1}
      const int d = c[k] == 0 ? (o[k] == 2 ? -1 : o[k]) : (c[k] == n - 1 ? (o[k] == 0 ? 1 : o[k] - 2) : o[k] - 1);
      const int w = c[k] + d;
      v[k] = w < 0 ? w + n : (w >= n ? w - n : w);
      const float x = pc[k] - floorf(pc[k] * g.inv_box[k]) * g.box[k];
      const float u = x - (float)c[k] * g.cell_len[k];
      const float gap = d == 0 ? 0.f : fmaxf(d > 0 ? g.cell_len[k] - u : u, 0.f);
      gap2 += gap * gap;
    }
    my_cell = (v[0] * g.nc[1] + v[1]) * g.nc[2] + v[2];
    culled = gap2 > a.cull2;
  }

  int* rad = a.rad + (int64_t)i * a.max_rad;
  int* ang = a.ang + (int64_t)i * a.max_ang;
  int* angpos = a.angpos + (int64_t)i * a.max_ang;
  int nr = 0, na = 0;   // list lengths so far (wavefront-uniform)
  bool overflow = false;
  // Accepted candidates are appended in lane order: a lane's place is the
  // number of accepting lanes below it.
  auto below = [](uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  };
  for (int s = 0; s < a.S; ++s) {
    if (lane == 0) {
      a.rad_off[(int64_t)i * (a.S + 1) + s] = nr;
      a.ang_off[(int64_t)i * (a.S + 1) + s] = na;
    }
    // candidate ranges of this species, one stencil cell per lane, and their prefix sums
    int st = 0, cnt = 0;
    if (lane < nst && !culled) {
      const int b = s * g.n_bins + my_cell;
      st = a.bin_start[b];
      cnt = a.bin_start[b + 1] - st;
    }
    int inc = cnt;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
      const int u = __shfl_up(inc, off, 64);
      if (lane >= off) inc += u;
    }
    const int total = __builtin_amdgcn_readfirstlane(__shfl(inc, nst - 1, 64));
    // one range (an open system): slots follow directly; short per-cell ranges
    // are flattened into LDS by their lanes; otherwise search the ranges
    const int st0 = __builtin_amdgcn_readfirstlane(st);
    const bool flat = nst > 1 && total <= kCandCap;
    __syncthreads();   // the previous species' candidates have been read
    if (lane < nst) {
      s_start[lane] = st;
      s_off[lane] = inc - cnt;
      if (flat)
        for (int q = 0; q < cnt; ++q) s_cand[inc - cnt + q] = st + q;
    }
    __syncthreads();
    // candidate slot at position c of the flattened sequence (-1 beyond it)
    auto candidate = [&](int c) {
      int j = -1;
      if (c < total) {
        if (nst == 1) {
          j = st0 + c;
        } else if (flat) {
          j = s_cand[c];
        } else {
          int lo = 0, hi = nst - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= c) lo = mid; else hi = mid - 1;
          }
          j = s_start[lo] + (c - s_off[lo]);
        }
      }
      return j;
    };
    // the next step's candidate and position are fetched before this step's
    // test, so the load is in flight while the wavefront works
    int j = candidate(lane);
    float4 pj = a.spos[j >= 0 && j != i ? j : i];
    for (int c0 = 0; c0 < total; c0 += 64) {
      const int jn = candidate(c0 + 64 + lane);
      const float4 pn = a.spos[jn >= 0 && jn != i ? jn : i];
      // straight-line test (invalid lanes read the centre's own position and
      // are masked), so the ballots take the comparison masks directly
      const bool valid = j >= 0 && j != i;
      const float r2 = pair_r2_exact(pi, pj, mi);
      const bool in_r = valid && r2 < a.rc2;
      const uint64_t mr = __builtin_amdgcn_ballot_w64(in_r);
      const int pr = nr + below(mr);
      // angular entries point into the radial list
      const bool in_a = valid && r2 < a.rca2 && pr < a.max_rad;
      const uint64_t ma = __builtin_amdgcn_ballot_w64(in_a);
      const int pa = na + below(ma);
      if (in_r && pr < a.max_rad) rad[(unsigned)pr] = j;
      if (in_a && pa < a.max_ang) {
        ang[(unsigned)pa] = j;
        angpos[(unsigned)pa] = pr;
      }
      nr += __popcll(mr);
      na += __popcll(ma);
      if (nr > a.max_rad || na > a.max_ang) {
        overflow = true;
        nr = min(nr, a.max_rad);
        na = min(na, a.max_ang);
      }
      j = jn;
      pj = pn;
    }
  }
  if (lane == 0) {
    a.rad_off[(int64_t)i * (a.S + 1) + a.S] = nr;
    a.ang_off[(int64_t)i * (a.S + 1) + a.S] = na;
    if (overflow) atomicOr(a.status, kStatusCapacity);
  }
}

// Same lists as k_neighbours, one wavefront per bin (periodic cell, or one
// system of a batch): the bin's centre atoms (all species, up to 64 at a
// time) are staged in LDS, and the stencil's candidates, one per lane and in
// ascending slot order, are tested against every centre in turn, each
// centre's accepted candidates being compacted with a ballot.  The stencil is
// set up once per bin instead of once per atom.  Per-centre list lengths live
// in the register of the lane with the centre's index.
__global__ __launch_bounds__(64) void k_neighbours_cell(NeighArgs a, Geometry g, int K) {
#pragma clang fp contract(off)
  __shared__ int s_start[kMaxStencil];
  __shared__ int s_off[kMaxStencil];
  __shared__ float4 s_cpos[64];
  __shared__ int s_cid[64];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int cell = b / K, part = b - cell * K;
  const int lane = threadIdx.x;
  const MinImage mi = min_image_of_system(g, cell);   // a batch's bins are its systems
  // stencil cells in ascending id order (see k_neighbours)
  int nst = 1;
  int my_cell = cell;
  if (g.periodic) {
    int c[3], nd[3], v[3][3];
    c[0] = cell / (g.nc[1] * g.nc[2]);
    c[1] = (cell / g.nc[2]) % g.nc[1];
    c[2] = cell % g.nc[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int n = g.nc[k];
      nd[k] = n >= 3 ? 3 : n;
      if (n >= 3) {
        if (c[k] == 0) { v[k][0] = 0; v[k][1] = 1; v[k][2] = n - 1; }
        else if (c[k] == n - 1) { v[k][0] = 0; v[k][1] = n - 2; v[k][2] = n - 1; }
        else { v[k][0] = c[k] - 1; v[k][1] = c[k]; v[k][2] = c[k] + 1; }
      } else {
        v[k][0] = 0; v[k][1] = 1; v[k][2] = 2;
      }
    }
    nst = nd[0] * nd[1] * nd[2];
    const int l = lane < nst ? lane : 0;
    const int o0 = l / (nd[1] * nd[2]), o1 = (l / nd[2]) % nd[1], o2 = l % nd[2];
    my_cell = (v[0][o0] * g.nc[1] + v[1][o1]) * g.nc[2] + v[2][o2];
  }

  // centre atoms of this cell (species-major ranges of slots); this wavefront
  // takes the part-th of K equal chunks of them
  int c_lo[kMaxSpecies], c_n[kMaxSpecies];
  int n_centres = 0;
#pragma unroll
  for (int s = 0; s < kMaxSpecies; ++s) {
    c_lo[s] = 0;
    c_n[s] = 0;
    if (s < a.S) {
      c_lo[s] = a.bin_start[s * g.n_bins + cell];
      c_n[s] = a.bin_start[s * g.n_bins + cell + 1] - c_lo[s];
      n_centres += c_n[s];
    }
  }
  const int chunk = (n_centres + K - 1) / K;
  const int q0 = part * chunk, q1 = min(n_centres, q0 + chunk);
  const uint64_t lt = __lanemask_lt();
  for (int cb = q0; cb < q1; cb += 64) {
    const int nc = min(64, q1 - cb);
    int my_i = -1;
    if (lane < nc) {
      int q = cb + lane, s = 0;
      while (q >= c_n[s]) { q -= c_n[s]; ++s; }
      my_i = c_lo[s] + q;
      s_cid[lane] = my_i;
      s_cpos[lane] = a.spos[my_i];
    }
    int nr = 0, na = 0;   // lists of centre `lane`
    bool overflow = false;
    for (int s = 0; s < a.S; ++s) {
      if (lane < nc) {
        a.rad_off[(int64_t)my_i * (a.S + 1) + s] = nr;
        a.ang_off[(int64_t)my_i * (a.S + 1) + s] = na;
      }
      int st = 0, cnt = 0;
      if (lane < nst) {
        const int bb = s * g.n_bins + my_cell;
        st = a.bin_start[bb];
        cnt = a.bin_start[bb + 1] - st;
      }
      int inc = cnt;
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        if (lane >= off) inc += u;
      }
      const int total = __shfl(inc, nst - 1, 64);
      __syncthreads();   // previous species' readers of s_start / s_off are done
      if (lane < nst) {
        s_start[lane] = st;
        s_off[lane] = inc - cnt;
      }
      __syncthreads();
      // candidate slot and position of the lane, one block of 64 ahead
      auto fetch = [&](int c, int& j, float4& pj) {
        j = -1;
        pj = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c < total) {
          int lo = 0, hi = nst - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= c) lo = mid; else hi = mid - 1;
          }
          j = s_start[lo] + (c - s_off[lo]);
          pj = a.spos[j];
        }
      };
      int jn;
      float4 pjn;
      fetch(lane, jn, pjn);
      for (int c0 = 0; c0 < total; c0 += 64) {
        const int j = jn;
        const float4 pj = pjn;
        if (c0 + 64 < total) fetch(c0 + 64 + lane, jn, pjn);
        for (int ci = 0; ci < nc; ++ci) {
          const float4 pi = s_cpos[ci];
          const int i = s_cid[ci];
          bool in_r = false, in_a = false;
          if (j >= 0 && j != i) {
            const float r2 = pair_r2_exact(pi, pj, mi);
            in_r = r2 < a.rc2;
            in_a = r2 < a.rca2;
          }
          const int base_r = __builtin_amdgcn_readlane(nr, ci);
          const int base_a = __builtin_amdgcn_readlane(na, ci);
          const uint64_t mr = __ballot(in_r);
          const int pr = base_r + __popcll(mr & lt);
          const bool in_a2 = in_a && pr < a.max_rad;
          const uint64_t ma = __ballot(in_a2);
          const int pa = base_a + __popcll(ma & lt);
          if (in_r && pr < a.max_rad) a.rad[(int64_t)i * a.max_rad + pr] = j;
          if (in_a2 && pa < a.max_ang) {
            a.ang[(int64_t)i * a.max_ang + pa] = j;
            a.angpos[(int64_t)i * a.max_ang + pa] = pr;
          }
          if (lane == ci) {
            nr += __popcll(mr);
            na += __popcll(ma);
            if (nr > a.max_rad || na > a.max_ang) {
              overflow = true;
              nr = min(nr, a.max_rad);
              na = min(na, a.max_ang);
            }
          }
        }
      }
    }
    if (lane < nc) {
      a.rad_off[(int64_t)my_i * (a.S + 1) + a.S] = nr;
      a.ang_off[(int64_t)my_i * (a.S + 1) + a.S] = na;
      if (overflow) atomicOr(a.status, kStatusCapacity);
    }
    __syncthreads();   // s_cid / s_cpos are rewritten by the next centre block
  }
}

// ---------------------------------------------------------------------------
// Neighbour lists from a pair list supplied by the caller (the MD engine's own
// list, a half list possibly with a buffer beyond the cutoff).  Each pair of
// NNP atoms is re-tested with the same FP32 predicate as the cell-list search
// and appended to both atoms' radial rows in arbitrary order; one wavefront
// per row then sorts it by slot (which groups it by species, slots being
// species-major), derives the species segments and the angular sub-list, so
// the lists are exactly the ones the cell-list search builds.
__device__ __forceinline__ float pair_r2(const float4& pi, const float4& pj, const Geometry& g) {
  return pair_r2_exact(pi, pj, min_image_of_system(g, 0));   // one system: the call's box or none
}

__global__ __launch_bounds__(kBlock) void k_pairs_scatter(const int* __restrict__ pairs, int n_pairs,
                                                          const int* __restrict__ loc, int n_atoms,
                                                          const int* __restrict__ islot,
                                                          const float4* __restrict__ spos, Geometry g, float rc2,
                                                          int* __restrict__ rad, int* __restrict__ pcount,
                                                          int max_rad, int* __restrict__ status) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const int a = pairs[2 * (int64_t)p], b = pairs[2 * (int64_t)p + 1];
  if (a < 0 || b < 0 || a >= n_atoms || b >= n_atoms || a == b) {
    atomicOr(status, kStatusInput);
    return;
  }
  const int la = loc[a], lb = loc[b];
  if (la < 0 || lb < 0) return;   // a pair with an atom outside the index group
  const int sa = islot[la], sb = islot[lb];
  if (!(pair_r2(spos[sa], spos[sb], g) < rc2)) return;
  const int pa = atomicAdd(&pcount[sa], 1), pb = atomicAdd(&pcount[sb], 1);
  if (pa < max_rad) rad[(int64_t)sa * max_rad + pa] = sb;
  if (pb < max_rad) rad[(int64_t)sb * max_rad + pb] = sa;
}

// Link atoms (eq. 4) are not atoms of the system, so a caller's pair list
// cannot name them: one wavefront per link atom tests it against every NNP
// atom with the same predicate and appends each pair within the cutoff to
// both rows.  A pair of two link atoms is added by the one with the lower
// index.  The NNP-local indices of the link atoms are [n - n_links, n).
__global__ __launch_bounds__(64) void k_link_pairs(int n, int n_links, const int* __restrict__ islot,
                                                   const float4* __restrict__ spos, Geometry g, float rc2,
                                                   int* __restrict__ rad, int* __restrict__ pcount, int max_rad) {
  const int tl = n - n_links + (int)blockIdx.x;
  const int sl = islot[tl];
  const float4 pl = spos[sl];
  for (int t = threadIdx.x; t < n; t += 64) {
    if (t >= n - n_links && t <= tl) continue;
    const int st = islot[t];
    if (!(pair_r2(pl, spos[st], g) < rc2)) continue;
    const int pa = atomicAdd(&pcount[sl], 1), pb = atomicAdd(&pcount[st], 1);
    if (pa < max_rad) rad[(int64_t)sl * max_rad + pa] = st;
    if (pb < max_rad) rad[(int64_t)st * max_rad + pb] = sl;
  }
}

// One wavefront per slot: bitonic sort of the row (padded to a power of two,
// at most kPairRowMax entries), then the species offsets and the angular list.
constexpr int kPairSort = kPairRowMax;

__global__ __launch_bounds__(64) void k_pairs_lists(NeighArgs a, Geometry g, const int* __restrict__ pcount) {
  __shared__ int row[kPairSort];
  __shared__ int arow[kPairSort];   // angular entries (slots), for the species counts
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const int cnt = pcount[i];
  bool overflow = cnt > a.max_rad;
  const int n = min(cnt, a.max_rad);
  int P = 64;
  while (P < n) P <<= 1;
  int* rrow = a.rad + (int64_t)i * a.max_rad;
  for (int t = lane; t < P; t += 64) row[t] = t < n ? rrow[t] : 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < P; t += 64) {
        const int u = t ^ j;
        if (u > t) {
          const int x = row[t], y = row[u];
          const bool up = (t & k) == 0;
          if ((x > y) == up) {
            row[t] = y;
            row[u] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  const float4 pi = a.spos[i];
  const uint64_t lt = __lanemask_lt();
  int* ang = a.ang + (int64_t)i * a.max_ang;
  int* angpos = a.angpos + (int64_t)i * a.max_ang;
  int na = 0;
  bool dup = false;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int t = c0 + lane;
    int j = -1;
    bool in_a = false;
    if (t < n) {
      j = row[t];
      rrow[t] = j;
      if (t > 0 && row[t - 1] == j) dup = true;
      in_a = pair_r2(pi, a.spos[j], g) < a.rca2;
    }
    const uint64_t ma = __ballot(in_a);
    const int pa = na + __popcll(ma & lt);
    if (in_a && pa < a.max_ang) {
      ang[pa] = j;
      angpos[pa] = t;
      arow[pa] = j;
    }
    na += __popcll(ma);
  }
  __syncthreads();
  if (na > a.max_ang) {
    overflow = true;
    na = a.max_ang;
  }
  // species segments: slots below each species' first slot
  if (lane <= a.S) {
    const int bound = lane < a.S ? a.bin_start[lane * g.n_bins] : 0x7fffffff;
    int r = 0, q = 0;
    for (int t = 0; t < n; ++t) r += row[t] < bound;
    for (int t = 0; t < na; ++t) q += arow[t] < bound;
    if (lane == a.S) { r = n; q = na; }
    a.rad_off[(int64_t)i * (a.S + 1) + lane] = r;
    a.ang_off[(int64_t)i * (a.S + 1) + lane] = q;
  }
  if (lane == 0 && overflow) atomicOr(a.status, kStatusCapacity);
  if (__ballot(dup) != 0 && lane == 0) atomicOr(a.status, kStatusInput);
}

inline int blocks_for(int64_t n, int b) { return (int)((n + b - 1) / b); }

// Smallest power of two PER <= kScanPerMax with nb <= kScanThreads * PER
// (kScanPerMax for larger histograms, which are scanned in several chunks).
inline int scan_entries_per_thread(int nb) {
  int per = 1;
  while (per < kScanPerMax && nb > kScanThreads * per) per *= 2;
  return per;
}

template <int PER>
void launch_scan(nnp_model& m, hipStream_t st) {
  const int nb = m.S * m.geo.n_bins;
  if (nb > kScanChunk) {   // many workgroups
    const int ca = (nb + kScanPartChunk - 1) / kScanPartChunk;
    const int cb = (m.geo.n_bins + kScanPartChunk - 1) / kScanPartChunk;
    hipLaunchKernelGGL(k_scan_part, dim3(ca + cb), dim3(kScanThreads), 0, st, m.d_bin_count, m.S, m.geo.n_bins, ca,
                       m.d_scan_part);
    hipLaunchKernelGGL(k_scan_fin, dim3(ca + cb), dim3(kScanThreads), 0, st, m.d_bin_count, m.d_bin_start,
                       m.d_cmstart, m.S, m.geo.n_bins, ca, m.d_scan_part);
    return;
  }
  hipLaunchKernelGGL(k_scan<PER>, dim3(1), dim3(kScanThreads), 0, st, m.d_bin_count, m.d_bin_start, m.d_cmstart,
                     m.S, m.geo.n_bins);
}

template <int PER>
void launch_cells_small(nnp_model& m, const float* pos, int n, const LinkArgs& L, hipStream_t st) {
  hipLaunchKernelGGL(k_cells_small<PER>, dim3(1), dim3(kScanThreads), 0, st, pos, n, m.d_idx, m.d_sigma, m.geo, L,
                     m.S, m.d_key, m.d_bin_start, m.d_perm, m.d_spos, m.d_slot_atom, m.d_order, m.d_sbin,
                     m.d_islot, m.d_pcount, m.d_status);
}

template <int PER>
void launch_scan_scatter(nnp_model& m, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_scatter<PER>, dim3(blocks_for(n, kScanThreads)), dim3(kScanThreads), 0, st,
                     m.d_bin_count, m.d_bin_start, m.d_cmstart, m.S, m.geo.n_bins, m.d_key, m.d_rank, n, m.d_tmp);
}

}  // namespace

hipError_t launch_cells(nnp_model& m, const float* pos, int n, hipStream_t st) {
  const Geometry& g = m.geo;
  LinkArgs L{m.d_link_ml, m.d_link_mm, m.link_d, m.n_links_dev};
  int nb = m.S * g.n_bins;
  if (n > 0 && g.periodic && n <= kSmallCells && nb <= kScanChunk) {
    switch (scan_entries_per_thread(nb)) {
      case 1: launch_cells_small<1>(m, pos, n, L, st); break;
      case 2: launch_cells_small<2>(m, pos, n, L, st); break;
      case 4: launch_cells_small<4>(m, pos, n, L, st); break;
      case 8: launch_cells_small<8>(m, pos, n, L, st); break;
      default: launch_cells_small<16>(m, pos, n, L, st); break;
    }
    return hipGetLastError();
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_stage, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, pos, n, m.d_idx,
                       m.d_sigma, m.d_sys, g, L, m.d_key, m.d_rank, m.d_stg, m.d_bin_count, m.d_status);
  }
  const bool fused = n > 0 && g.periodic && nb <= kScanChunk;
  const int per = scan_entries_per_thread(nb);
  if (fused) {
    switch (per) {
      case 1: launch_scan_scatter<1>(m, n, st); break;
      case 2: launch_scan_scatter<2>(m, n, st); break;
      case 4: launch_scan_scatter<4>(m, n, st); break;
      case 8: launch_scan_scatter<8>(m, n, st); break;
      default: launch_scan_scatter<16>(m, n, st); break;
    }
  } else {
    switch (per) {
      case 1: launch_scan<1>(m, st); break;
      case 2: launch_scan<2>(m, st); break;
      case 4: launch_scan<4>(m, st); break;
      case 8: launch_scan<8>(m, st); break;
      default: launch_scan<16>(m, st); break;
    }
  }
  if (n > 0 && !g.periodic) {
    hipLaunchKernelGGL(k_rank_systems, dim3(g.n_bins), dim3(64), 0, st, m.d_sys_off, g.n_bins, m.S, m.d_bin_start,
                       m.d_sigma, m.d_idx, pos, g, L, m.d_cmstart, m.d_perm, m.d_spos, m.d_slot_atom,
                       m.d_order, m.d_bin_count, m.d_sbin, m.d_islot, m.d_pcount);
  } else if (n > 0) {
    if (!fused)
      hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, m.d_key, m.d_rank, n,
                         m.d_bin_start, m.d_tmp);
    hipLaunchKernelGGL(k_binsort, dim3(blocks_for((int64_t)nb * 64, kBlock)), dim3(kBlock), 0, st,
                       m.d_bin_start, nb, m.d_tmp, m.d_stg, m.d_idx, g, m.d_cmstart, m.S, m.d_perm,
                       m.d_spos, m.d_slot_atom, m.d_order, m.d_sbin, m.d_islot, m.d_pcount, m.d_bin_count);
  }
  return hipGetLastError();
}

// Wavefronts per cell share the candidate loads and the stencil set-up among
// a few centre atoms each; that wins on large periodic grids (98k atoms:
// 114 us against 156 us per atom), one wavefront per atom on smaller ones
// (12k atoms: 32 us against 36 us) and for open systems.  A pinned or tuned
// choice overrides the default.
int neighbour_variant(const nnp_model& m, int n) {
  if (m.geo.n_bins < 2) return 0;
  const int v = stage_variant(m, kTuneNeighbours, n);
  return v >= 0 ? v : 0;
}

hipError_t launch_neighbours(nnp_model& m, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  NeighArgs a;
  a.order = m.d_order;
  a.sbin = m.d_sbin;
  a.spos = m.d_spos;
  a.perm = m.d_perm;
  a.key = m.d_key;
  a.bin_start = m.d_bin_start;
  a.n = n;
  a.S = m.S;
  a.rc2 = m.dp.rc_rad * m.dp.rc_rad;
  a.rca2 = m.dp.rc_ang * m.dp.rc_ang;
  {
    const float rm = std::sqrt(a.rc2) + kCullMargin;
    a.cull2 = rm * rm;
  }
  a.rad = m.d_nbr_rad;
  a.ang = m.d_nbr_ang;
  a.angpos = m.d_angpos;
  a.rad_off = m.d_rad_off;
  a.ang_off = m.d_ang_off;
  a.max_rad = m.max_rad;
  a.max_ang = m.max_ang;
  a.status = m.d_status;
  const int v = neighbour_variant(m, n);
  if (v >= 1) {
    // K wavefronts share a cell, each with about 8 / 5 / 3 centre atoms
    const int target = v == 1 ? 8 : (v == 2 ? 5 : 3);
    const int per_bin = (n + m.geo.n_bins - 1) / m.geo.n_bins;
    const int K = std::max(1, std::min(16, (per_bin + target - 1) / target));
    hipLaunchKernelGGL(k_neighbours_cell, dim3((unsigned)(m.geo.n_bins * K)), dim3(64), 0, st, a, m.geo, K);
  } else {
    hipLaunchKernelGGL(k_neighbours, dim3(n), dim3(64), 0, st, a, m.geo);
  }
  return hipGetLastError();
}

hipError_t launch_pair_lists(nnp_model& m, int n, int n_atoms, int n_pairs, const int* pairs, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (n_pairs > 0) {
    hipLaunchKernelGGL(k_pairs_scatter, dim3(blocks_for(n_pairs, kBlock)), dim3(kBlock), 0, st, pairs, n_pairs,
                       m.d_loc, n_atoms, m.d_islot, m.d_spos, m.geo, m.dp.rc_rad * m.dp.rc_rad, m.d_nbr_rad,
                       m.d_pcount, m.max_rad, m.d_status);
  }
  if (m.n_links_dev > 0) {
    hipLaunchKernelGGL(k_link_pairs, dim3(m.n_links_dev), dim3(64), 0, st, n, m.n_links_dev, m.d_islot, m.d_spos,
                       m.geo, m.dp.rc_rad * m.dp.rc_rad, m.d_nbr_rad, m.d_pcount, m.max_rad);
  }
  NeighArgs a;
  a.order = m.d_order;
  a.sbin = m.d_sbin;
  a.spos = m.d_spos;
  a.perm = m.d_perm;
  a.key = m.d_key;
  a.bin_start = m.d_bin_start;
  a.n = n;
  a.S = m.S;
  a.rc2 = m.dp.rc_rad * m.dp.rc_rad;
  a.rca2 = m.dp.rc_ang * m.dp.rc_ang;
  {
    const float rm = std::sqrt(a.rc2) + kCullMargin;
    a.cull2 = rm * rm;
  }
  a.rad = m.d_nbr_rad;
  a.ang = m.d_nbr_ang;
  a.angpos = m.d_angpos;
  a.rad_off = m.d_rad_off;
  a.ang_off = m.d_ang_off;
  a.max_rad = m.max_rad;
  a.max_ang = m.max_ang;
  a.status = m.d_status;
  hipLaunchKernelGGL(k_pairs_lists, dim3(n), dim3(64), 0, st, a, m.geo, m.d_pcount);
  return hipGetLastError();
}

}  // namespace nnp
