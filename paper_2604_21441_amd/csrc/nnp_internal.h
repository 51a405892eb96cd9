// Internal declarations of the NNP library: model state, kernel parameter
// blocks and the launchers of each stage.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <map>
#include <utility>
#include <vector>

#include "nnp.h"

namespace nnp {

constexpr int kRadShifts = 16;   // radial shifts per species
constexpr int kAngShifts = 8;    // angular radial shifts per species pair
constexpr int kAngSects = 4;     // angle sections per species pair
constexpr int kMaxSpecies = 4;
constexpr int kMaxPairs = kMaxSpecies * (kMaxSpecies + 1) / 2;
constexpr int kTileAtoms = 16;   // atoms of the smallest network tile (sizes the energy partials)

// Stages with several kernel variants chosen by the autotuner.
enum TuneStage { kTuneNeighbours = 0, kTuneDescriptor = 1, kTuneNetwork = 2, kTuneAdjoint = 3, kTuneStages = 4 };

// Workgroups are dispatched round-robin over the XCDs, each with its own L2.
// xcd_block renumbers them so that every XCD works through one contiguous
// range of the visiting order (a bijection of [0, G)); correctness never
// depends on it.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int q = G / kXcds, r = G % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Cross-lane sums with DPP row permutations (VALU operands, no LDS round
// trip): mirror (l <-> 15-l), half-mirror (l <-> 7-l within each half) and
// the quad swaps xor 2 and xor 1 pair the lanes of a 16-lane row disjointly.
constexpr int kDppMirror = 0x140;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppXor2 = 0x4E;       // quad_perm(2, 3, 0, 1)
constexpr int kDppXor1 = 0xB1;       // quad_perm(1, 0, 3, 2)

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// One step of a transposing butterfly: v[0, 2H) -> v[0, H), keeping the half
// selected by `upper` and adding the partner's copy of that half.
template <int H, int CTRL>
__device__ __forceinline__ void halve(float* v, bool upper) {
#pragma unroll
  for (int e = 0; e < H; ++e) {
    const float keep = upper ? v[e + H] : v[e];
    const float send = upper ? v[e] : v[e + H];
    v[e] = keep + dpp<CTRL>(send);
  }
}

// Mixed network tiling: the species with the fewest atoms (lowest index on
// ties; empty species are skipped) takes tiles of 16 atoms, the others the
// kernel's full width, so that a small system splits into workgroups of more
// even size.  -1 when there is a single species.  The network kernel and the energy reduction both call it
// on the same bucket boundaries, so they agree on the tile count.
__device__ __forceinline__ int narrow_species(const int* bin_start, int S, int n_bins) {
  if (S < 2) return -1;
  int best = -1, fewest = 0x7fffffff;
  for (int s = 0; s < S; ++s) {
    const int c = bin_start[(s + 1) * n_bins] - bin_start[s * n_bins];
    if (c > 0 && c < fewest) {
      fewest = c;
      best = s;
    }
  }
  return best;
}

// Device status bits.
constexpr int kStatusCapacity = 1;
constexpr int kStatusNonFinite = 2;
constexpr int kStatusInput = 4;      // bad entry in a caller's pair list
constexpr int kPairRowMax = 256;     // radial capacity the pair-list sort supports

// Descriptor constants, passed by value to the kernels.
struct DescParams {
  float rc_rad, rc_ang;
  float eta_rad, eta_ang, zeta;
  float ang_pref;                       // 2^(1 - zeta)
  float rad_shift[kRadShifts];
  float ang_shift[kAngShifts];
  float cos_sect[kAngSects], sin_sect[kAngSects];
  // Pre-scaled forms used by the row kernels: exp(-eta (r - Rs)^2) =
  // exp2(-(r sq - Rs sq)^2) with sq = sqrt(eta log2 e); the angular mean
  // distance enters as r_j hq + r_k hq with hq = sq / 2; sq_pref^2 = 2^(1-zeta).
  float sq_eta_r, hq_eta_a, sq_pref;
  float rad_shift_s[kRadShifts], ang_shift_s[kAngShifts];
  // Derived FP32 constants, computed once on the host with the same IEEE
  // operations the kernels would use: 1/(2 Rc) and 1/(2 Rca) (cos(pi r / Rc) =
  // cos of r/(2 Rc) revolutions), -pi/(2 Rc) and -pi/(2 Rca) (the cutoff
  // derivative factor), -2 eta_r / sq_eta_r and -eta_a / hq_eta_a (the chain
  // factors of the scaled Gaussians in the adjoint).
  float inv2rc, inv2rca, dfc_r, dfc_a, c1_rad, c_sdr;
  uint64_t class_tab;                   // class of species pair (a, b) in bits 4 (4 a + b) .. +3
  float mm_cutoff, ke;
  int S, P, D, stride;                  // species, pair classes, descriptor length, row stride
  int extra;                            // 1 if the MM potential is the last input
  int pair_a[kMaxPairs], pair_b[kMaxPairs];
  int class_of[kMaxSpecies][kMaxSpecies];  // unordered species pair -> class
};

// Geometry of the current call.
struct Geometry {
  int periodic;                         // 1: one orthorhombic box, minimum image, cell grid
  float box[3], inv_box[3];
  int nc[3];                            // cells per dimension (periodic)
  float cell_scale[3];                  // nc * (1/L) in FP32
  float cell_len[3];                    // L / nc in FP32
  int n_bins;                           // cells (periodic) or systems (batched)
  // Batched calls with per-system boxes (periodic = 0, bins are systems):
  // sys_box[2 s] = (L_x, L_y, L_z, 0) and sys_box[2 s + 1] = (1/L_x, 1/L_y,
  // 1/L_z, 0) in FP32, zeros for an open system; sbin[slot] = system.  Null
  // otherwise.
  const float4* sys_box;
  const int* sbin;
};

// Minimum-image lengths for the pairs of one centre atom: the call's box,
// the box of the centre's system in a batch, or none (on = false).
struct MinImage {
  float L[3], iL[3];
  bool on;
};

__device__ __forceinline__ MinImage min_image_of_system(const Geometry& g, int sys) {
  MinImage b;
  if (g.sys_box) {
    const float4 lo = g.sys_box[2 * sys], hi = g.sys_box[2 * sys + 1];
    b.L[0] = lo.x; b.L[1] = lo.y; b.L[2] = lo.z;
    b.iL[0] = hi.x; b.iL[1] = hi.y; b.iL[2] = hi.z;
    b.on = lo.x > 0.f;
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      b.L[k] = g.box[k];
      b.iL[k] = g.inv_box[k];
    }
    b.on = g.periodic != 0;
  }
  return b;
}

__device__ __forceinline__ MinImage min_image_at(const Geometry& g, int slot) {
  return min_image_of_system(g, g.sys_box ? g.sbin[slot] : 0);
}

// r^2 of d = pj - pi under the minimum image, every operation one IEEE FP32
// operation in a fixed order (no contraction): the neighbour predicate of the
// cell list and the pair lists.
__device__ __forceinline__ float pair_r2_exact(const float4& pi, const float4& pj, const MinImage& b) {
#pragma clang fp contract(off)
  float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
  if (b.on) {
    float sx = rintf(dx * b.iL[0]);
    float sy = rintf(dy * b.iL[1]);
    float sz = rintf(dz * b.iL[2]);
    float tx = sx * b.L[0], ty = sy * b.L[1], tz = sz * b.L[2];
    dx = dx - tx; dy = dy - ty; dz = dz - tz;
  }
  float xx = dx * dx, yy = dy * dy, zz = dz * dz;
  float r2 = xx + yy;
  return r2 + zz;
}
// Cells per dimension are capped so that a cell's coordinates pack into
// 10 bits each (larger cells stay correct).
constexpr int kMaxCellsPerDim = 1023;

// Link atoms: NNP-local atoms t >= n_group have idx[t] = -1 - l.
struct LinkArgs {
  const int* ml;     // [n_links] ML atom index
  const int* mm;     // [n_links] MM atom index
  float d;
  int n;
};

// Neighbour-list arrays (per sorted slot).
struct NbrLists {
  int* rad;      // [n][max_rad]
  int* ang;      // [n][max_ang]
  int* rad_off;  // [n][S+1] segment starts by species within the row
  int* ang_off;  // [n][S+1]
  int max_rad, max_ang;
};

// Network tile schedule: species buckets are bins [s*n_bins, (s+1)*n_bins).
struct MlpArgs {
  const float* x;          // [n][stride]
  float* g;                // [n][stride]  dE/dx (output)
  float* e;                // [n] atomic energies (output)
  const void* wmat;        // fragment-packed matrices (FP32 or BF16)
  const float* wvec;       // biases and output weights (FP32)
  const int* bin_start;    // species bucket boundaries
  int n_bins, S, n_members, stride;
  int64_t mat_per_species; // elements per (member, species) in wmat
  int64_t vec_per_species; // elements per (member, species) in wvec
  double* part;            // per-wavefront FP64 energy partials, or null
  int* status;
  float* q;                // predicted atomic charges (output), or null: no charge head
  int phi_col;             // column of x holding the MM potential (models with charges)
  const void* wrow;        // BF16 models: W1, W2, W3 row-major per (member, species), or null
  int64_t wrow_per_species;
};

// Per-call device workspace: capacities and the arrays sized from them.
// nnp_reserve carves it out of one allocation; the no-allocation entry
// point carves the same layout out of a static device array for one call.
struct Workspace {
  // capacities
  int max_atoms = 0, max_sys = 0, max_mm = 0, max_rad = 0, max_ang = 0, max_bins = 0;

  // device arrays
  int* d_idx = nullptr;        // NNP-local atom -> atom index
  int* d_sigma = nullptr;      // NNP-local atom -> species
  int* d_sys = nullptr;        // NNP-local atom -> system (batched)
  int* d_sys_off = nullptr;    // [n_sys + 1] first NNP-local atom of each open system
  int* d_key = nullptr;
  int* d_bin_count = nullptr;
  int* d_bin_start = nullptr;  // [max_bins + 1]
  int* d_cmstart = nullptr;    // [max_bins] bin-major starts (bin * S + species)
  int* d_scan_part = nullptr;  // chunk totals of the many-workgroup histogram scan
  int* d_order = nullptr;      // [max_atoms] slots in bin-major visiting order
  int* d_perm = nullptr;       // slot -> NNP-local atom
  int* d_tmp = nullptr;        // scatter order before the in-bin ranking
  int* d_rank = nullptr;       // arrival rank of each atom among the atoms of its bin key
  float4* d_spos = nullptr;    // slot -> position (w = species bits)
  float4* d_stg = nullptr;     // NNP-local atom -> staged position (w = species bits)
  int* d_slot_atom = nullptr;  // slot -> atom index
  int* d_sbin = nullptr;       // slot -> cell coordinates x<<20 | y<<10 | z (periodic) or system
  int* d_loc = nullptr;        // system atom -> NNP-local index or -1 (pair lists)
  int* d_islot = nullptr;      // NNP-local index -> slot
  int* d_pcount = nullptr;     // radial entries per slot while a pair list is scattered
  int* d_nbr_rad = nullptr;
  int* d_nbr_ang = nullptr;
  int* d_rad_off = nullptr;
  int* d_ang_off = nullptr;
  int* d_angpos = nullptr;     // [n][max_ang] position of each angular neighbour in the radial list
  float3* d_contrib = nullptr; // [n][max_rad] force on atom i from the centre at its radial slot
  double* d_self = nullptr;    // [n][3] force on each atom from its own environment
  double* d_part = nullptr;    // per-wavefront FP64 energy partials
  int max_part = 0;
  float* d_x = nullptr;
  float* d_g = nullptr;
  float* d_e = nullptr;
  float* d_mm_part = nullptr;  // MM channel per-workgroup partials [mm_partial_floats(max_atoms, max_mm)]
  float* d_q = nullptr;        // predicted atomic charges (member mean) [max_atoms], models with charges
  float4* d_sys_box = nullptr; // [2 max_sys] per-system boxes of a batched call (Geometry::sys_box)
};

}  // namespace nnp

// The model object.
struct nnp_model : nnp::Workspace {
  int device = 0;
  int n_cu = 256;                       // compute units of the device
  nnp_precision prec = NNP_FP32;
  int S = 0, P = 0, D = 0, Din = 0, stride = 0, n_members = 1, extra = 0;
  int charges = 0;                      // second network output: an atomic charge in the MM potential
  std::vector<int> species;             // atomic numbers, ascending
  std::vector<int> widths;              // unpadded widths
  float celu_alpha = 0.1f;
  nnp::DescParams dp{};
  int mlp_cols = 1;                     // column tiles (16 atoms each) per network workgroup
  int mlp_mixed = 0;                    // the species with the fewest atoms uses one column tile
  std::map<std::pair<int, int>, int> tuned;   // (stage, size bucket) -> variant
  int force_variant[nnp::kTuneStages] = {-1, -1, -1, -1};   // set while timing candidates
  int pinned[nnp::kTuneStages] = {-1, -1, -1, -1};          // nnp_set_variant
  int net_kind = 0;                     // 0 water (128-160-128-96), 1 hcno (384/416-256-192-160)
  std::vector<float> w_host;            // canonical FP32 weights, draw order

  // device weights
  void* d_wmat = nullptr;
  float* d_wvec = nullptr;
  void* d_wrow = nullptr;               // BF16: W1, W2, W3 row-major (the LDS-resident network kernel)
  int64_t wrow_per_species = 0;         // elements per (member, species) in d_wrow
  int64_t mat_per_species = 0, vec_per_species = 0;

  bool reserved = false;
  void* d_ws_base = nullptr;    // the one allocation every Workspace array of nnp_reserve lives in
  int* d_status = nullptr;
  int* h_stage = nullptr;      // pinned staging for topology uploads

  // link atoms
  std::vector<int> link_ml, link_mm;
  float link_d = 1.0f;
  int link_Z = 1, link_sigma = 0, link_version = 0;
  int* d_link_ml = nullptr;
  int* d_link_mm = nullptr;
  double* d_link_F = nullptr;  // [n_links][3] force on each link atom
  int n_links_dev = 0;

  // topology cache (host copies)
  int topo_mode = -1;          // 0 single system, 1 batched
  int topo_n_atoms = -1;
  int topo_link_version = -1;
  std::vector<int> topo_Z, topo_idx, topo_offsets;
  std::vector<float> topo_boxes;       // per-system boxes of the last batched call as uploaded ([n_sys][8])
  int n_nnp = 0;

  // graph replay of identical calls
  bool graph_enabled = true;
  hipStream_t cap_stream = nullptr;  // capture stream (default priority)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint8_t> graph_key;
  int64_t graph_replays = 0;           // launches of an unchanged graph
  int64_t graph_updates = 0;           // graphs updated in place for a call with new arguments
  int64_t graph_builds = 0;            // graphs instantiated

  // stage timing
  std::vector<hipEvent_t> prof_ev;   // [call][stage][2]
  int prof_max_calls = 0, prof_calls = 0;

  // last call
  nnp::Geometry geo{};
  int last_n = 0;
};

namespace nnp {

// autotuner (api.cpp): tuned variant of a stage for n atoms, or -1
int tuned_choice(const nnp_model& m, int stage, int n);
int descriptor_variant(const nnp_model& m, int n);
int neighbour_variant(const nnp_model& m, int n);
int mlp_variant(const nnp_model& m, int n);
int adjoint_variant(const nnp_model& m, int n);
// Variant of a tuned stage: the candidate being timed, else the pinned one,
// else the tuned choice for this size; -1 means the stage's default.
int stage_variant(const nnp_model& m, int stage, int n);
constexpr int kStageVariants[kTuneStages] = {4, 5, 10, 3};
// Histograms of more than this many entries are scanned by many workgroups
// (chunk totals, then each chunk with the sum of the earlier ones).
constexpr int kScanPartChunk = 4096;
int size_bucket(int n);

// workspace (api.cpp): capacities for a call of up to max_atoms atoms, and the
// layout of every array at 256-byte aligned offsets from base (null: measure
// only); returns the bytes the layout spans.
Workspace workspace_caps(const nnp_model& m, int max_atoms, int max_systems, int max_mm, int max_rad, int max_ang);
size_t carve_workspace(const nnp_model& m, Workspace& w, char* base);
// geometry and the stage sequence of one call (api.cpp)
nnp_status setup_periodic(nnp_model* m, const float* box);
nnp_status run_path(nnp_model* m, int n, const float* pos, int n_mm, const float* mm_pos, const float* mm_q,
                    double* energies, int n_sys, double* forces, double* mm_forces, int accumulate,
                    int assign_forces, int n_atoms, int n_pairs, const int* pairs, hipStream_t st);

// noalloc.hip: size of the static workspace of nnp_compute_noalloc, and the
// once-per-device lookup of its device address (called by nnp_create)
constexpr size_t kNoallocScratchBytes = size_t(32) << 20;
nnp_status noalloc_scratch_setup(int device);

// error helpers (api.cpp)
nnp_status set_error(nnp_status s, const std::string& msg);
nnp_status hip_error(hipError_t e, const char* what);

// weights.cpp
void draw_weights(uint64_t seed, const std::vector<int>& widths, int n_species, int n_members,
                  std::vector<float>& out);
void pack_weights(const nnp_model& m, std::vector<uint8_t>& mat, std::vector<float>& vec,
                  int64_t& mat_per_species, int64_t& vec_per_species);
// BF16 (round to nearest even) copies of W1 [N1 x K0p] (zero columns beyond the
// real input width), W2 [N2 x N1] and W3 [N3 x N2], row-major, per (member, species).
void pack_rows_bf16(const nnp_model& m, std::vector<uint16_t>& out, int64_t& per_species);

// cells.hip
hipError_t launch_cells(nnp_model& m, const float* pos, int n_nnp, hipStream_t st);
hipError_t launch_neighbours(nnp_model& m, int n_nnp, hipStream_t st);
hipError_t launch_pair_lists(nnp_model& m, int n, int n_atoms, int n_pairs, const int* pairs, hipStream_t st);

// descriptor.hip
hipError_t launch_descriptor_fwd(nnp_model& m, int n, hipStream_t st);
hipError_t launch_descriptor_bwd(nnp_model& m, int n, hipStream_t st);
hipError_t launch_force_gather(nnp_model& m, int n, double* forces, int assign, double* energies, int n_sys,
                               int accumulate, hipStream_t st);

// mm.hip
size_t mm_partial_floats(int max_atoms, int max_mm);   // floats of the MM partial buffer
hipError_t launch_mm_fwd(nnp_model& m, int n, int n_mm, const float* mm_pos, const float* mm_q,
                         hipStream_t st);
hipError_t launch_mm_bwd(nnp_model& m, int n, int n_mm, const float* mm_pos, const float* mm_q,
                         double* forces, double* mm_forces, hipStream_t st);

// mlp.hip
hipError_t launch_mlp(nnp_model& m, int n, hipStream_t st);

// fills (api.cpp)
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t st);
hipError_t launch_me_pairs(int n_ml, const float* ml_pos, const float* ml_par, int n_mm, const float* mm_pos,
                           const float* mm_par, const Geometry& g, float cutoff, float ke, double* energy,
                           double* ml_f, double* mm_f, int accumulate, hipStream_t st);
hipError_t launch_link_redistribute(nnp_model& m, const float* pos, double* forces, hipStream_t st);

}  // namespace nnp
