// C ABI entry points: model lifecycle, argument validation, the topology
// cache, and the per-call sequence of stage launches on the caller's stream.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "nnp_internal.h"

namespace nnp {

static thread_local std::string g_last_error;

nnp_status set_error(nnp_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

nnp_status hip_error(hipError_t e, const char* what) {
  return set_error(NNP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int size_bucket(int n) {
  // quarter-octave buckets of the atom count
  return n <= 1 ? 0 : (int)std::lround(4.0 * std::log2((double)n));
}

int tuned_choice(const nnp_model& m, int stage, int n) {
  auto it = m.tuned.find({stage, size_bucket(n)});
  return it == m.tuned.end() ? -1 : it->second;
}

int stage_variant(const nnp_model& m, int stage, int n) {
  if (m.force_variant[stage] >= 0) return m.force_variant[stage];
  if (m.pinned[stage] >= 0) return m.pinned[stage];
  return tuned_choice(m, stage, n);
}

Workspace workspace_caps(const nnp_model& m, int max_atoms, int max_systems, int max_mm, int max_rad,
                         int max_ang) {
  Workspace w;
  w.max_atoms = max_atoms;
  w.max_sys = max_systems;
  w.max_mm = max_mm;
  w.max_rad = max_rad;
  w.max_ang = max_ang;
  const int cells_cap = max_atoms > 64 ? max_atoms : 64;
  const int per_species_bins = cells_cap > max_systems ? cells_cap : max_systems;
  w.max_bins = m.S * per_species_bins;
  w.max_part = max_atoms / kTileAtoms + 2 * kMaxSpecies + 8;
  return w;
}

// Every array of the workspace at its own 256-byte aligned offset from `base`
// (a null base only measures).  The pointers are written into w.
size_t carve_workspace(const nnp_model& m, Workspace& w, char* base) {
  size_t off = 0;
  auto take = [&](auto*& p, size_t count) {
    using T = std::remove_reference_t<decltype(*p)>;
    off = (off + 255) & ~size_t(255);
    p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (count ? count : 1) * sizeof(T);
  };
  const size_t n = (size_t)w.max_atoms;
  take(w.d_idx, n);
  take(w.d_sigma, n);
  take(w.d_sys, n);
  take(w.d_sys_off, (size_t)w.max_sys + 2);
  take(w.d_key, n);
  take(w.d_perm, n);
  take(w.d_tmp, n);
  take(w.d_rank, n);
  take(w.d_slot_atom, n);
  take(w.d_sbin, n);
  take(w.d_loc, n);
  take(w.d_islot, n);
  take(w.d_pcount, n);
  take(w.d_spos, n);
  take(w.d_stg, n);
  take(w.d_bin_count, (size_t)w.max_bins);
  take(w.d_bin_start, (size_t)w.max_bins + 1);
  take(w.d_cmstart, (size_t)w.max_bins);
  take(w.d_scan_part, 2 * ((size_t)w.max_bins / kScanPartChunk + 2));
  take(w.d_order, n);
  take(w.d_nbr_rad, n * w.max_rad);
  take(w.d_nbr_ang, n * w.max_ang);
  take(w.d_rad_off, n * (m.S + 1));
  take(w.d_ang_off, n * (m.S + 1));
  take(w.d_angpos, n * w.max_ang);
  take(w.d_contrib, n * w.max_rad);
  take(w.d_self, 3 * n);
  take(w.d_part, (size_t)w.max_part);
  take(w.d_x, n * m.stride);
  take(w.d_g, n * m.stride);
  take(w.d_e, n);
  w.d_mm_part = nullptr;
  if (m.extra && w.max_mm > 0) take(w.d_mm_part, mm_partial_floats(w.max_atoms, w.max_mm));
  w.d_q = nullptr;
  if (m.charges) take(w.d_q, n);
  take(w.d_sys_box, 2 * (size_t)w.max_sys);
  return (off + 255) & ~size_t(255);
}

namespace {

#define HIP_TRY(expr, what)                      \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_error(e_, what); \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void drop_graph(nnp_model* m) {
  if (m->graph_exec) (void)hipGraphExecDestroy(m->graph_exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->graph_exec = nullptr;
  m->graph = nullptr;
  m->graph_key.clear();
}

// Byte image of everything a captured sequence depends on besides device
// memory contents: pointers, sizes, flags and the geometry passed by value.
template <typename... T>
std::vector<uint8_t> make_key(const T&... parts) {
  std::vector<uint8_t> k;
  auto add = [&](const auto& v) {
    const uint8_t* b = reinterpret_cast<const uint8_t*>(&v);
    k.insert(k.end(), b, b + sizeof(v));
  };
  (add(parts), ...);
  return k;
}

// Run `launch(stream)` directly, or replay / capture it as a HIP graph.
// Identical calls (same key) replay one graph: one launch instead of ~15.
// A call with another key (a new box, other output buffers) captures its
// launches again and first tries to update the instantiated graph in place
// (hipGraphExecUpdate: same kernels in the same order, new arguments), which
// is far cheaper than instantiating; only if that fails is the graph rebuilt.
// Capture happens on the model's own stream (the caller's may be the legacy
// default stream, which cannot be captured); the graph runs on the caller's.
template <typename F>
nnp_status dispatch(nnp_model* m, std::vector<uint8_t> key, hipStream_t st, F launch) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (!m->graph_enabled || !m->cap_stream || m->prof_calls < m->prof_max_calls ||
      (st != nullptr && (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone))) {
    return launch(st);
  }
  if (m->graph_exec && key == m->graph_key) {
    HIP_TRY(hipGraphLaunch(m->graph_exec, st), "graph replay");
    ++m->graph_replays;
    return NNP_OK;
  }
  HIP_TRY(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal), "graph capture");
  nnp_status s = launch(m->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(m->cap_stream, &g);
  if (s != NNP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return hip_error(e, "graph capture");
  if (m->graph_exec) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateError;
    if (hipGraphExecUpdate(m->graph_exec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
      if (m->graph) (void)hipGraphDestroy(m->graph);
      m->graph = g;
      m->graph_key = std::move(key);
      ++m->graph_updates;
      HIP_TRY(hipGraphLaunch(m->graph_exec, st), "graph launch");
      return NNP_OK;
    }
    (void)hipGetLastError();
  }
  drop_graph(m);
  e = hipGraphInstantiate(&m->graph_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    m->graph_exec = nullptr;
    return hip_error(e, "graph instantiate");
  }
  m->graph = g;
  m->graph_key = std::move(key);
  ++m->graph_builds;
  HIP_TRY(hipGraphLaunch(m->graph_exec, st), "graph launch");
  return NNP_OK;
}

void free_workspace(nnp_model* m) {
  if (m->d_ws_base) (void)hipFree(m->d_ws_base);
  m->d_ws_base = nullptr;
  static_cast<Workspace&>(*m) = Workspace{};
  if (m->h_stage) (void)hipHostFree(m->h_stage);
  m->h_stage = nullptr;
  m->reserved = false;
  m->topo_mode = -1;
  m->topo_boxes.clear();
  drop_graph(m);
}

int descriptor_length(int S) { return kRadShifts * S + kAngShifts * kAngSects * (S * (S + 1) / 2); }

// Upload host topology data (n 4-byte words) through the pinned staging
// buffer, ordered after the stream's earlier work.  This synchronises the
// stream, so it is refused while the stream is being captured.
nnp_status upload_words(nnp_model* m, void* dst, const void* src, int n, hipStream_t st) {
  if (n <= 0) return NNP_OK;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (st != nullptr && (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone))
    return set_error(NNP_ESTATE,
                     "a new topology (atomic numbers, index group, offsets or batch boxes) cannot be uploaded while "
                     "the stream is being captured: make one call with it outside the capture first");
  std::memcpy(m->h_stage, src, 4 * (size_t)n);
  HIP_TRY(hipMemcpyAsync(dst, m->h_stage, 4 * (size_t)n, hipMemcpyHostToDevice, st), "topology upload");
  HIP_TRY(hipStreamSynchronize(st), "topology upload");
  return NNP_OK;
}

nnp_status upload_ints(nnp_model* m, int* dst, const int* src, int n, hipStream_t st) {
  return upload_words(m, dst, src, n, st);
}

nnp_status species_of(const nnp_model* m, int z, int* out) {
  for (int s = 0; s < m->S; ++s)
    if (m->species[s] == z) {
      *out = s;
      return NNP_OK;
    }
  return set_error(NNP_ESPECIES, "atomic number " + std::to_string(z) + " is not in the species table");
}

// Tuning cache file (NNP_TUNE_CACHE): one line per entry,
// "<arch> <network kind> <precision> <stage> <size bucket> <variant>".
std::string device_arch(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

void load_tuning(nnp_model* m) {
  const char* path = std::getenv("NNP_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  const std::string arch = device_arch(m->device);
  char a[64];
  int kind, prec, stage, bucket, variant;
  while (std::fscanf(f, "%63s %d %d %d %d %d", a, &kind, &prec, &stage, &bucket, &variant) == 6)
    if (arch == a && kind == m->net_kind && prec == (int)m->prec && stage >= 0 && stage < kTuneStages)
      m->tuned[{stage, bucket}] = variant;
  std::fclose(f);
}

void save_tuning(const nnp_model* m) {
  const char* path = std::getenv("NNP_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  const std::string arch = device_arch(m->device);
  for (const auto& kv : m->tuned)
    std::fprintf(f, "%s %d %d %d %d %d\n", arch.c_str(), m->net_kind, (int)m->prec, kv.first.first, kv.first.second,
                 kv.second);
  std::fclose(f);
}

}  // namespace
}  // namespace nnp

using namespace nnp;

extern "C" {

const char* nnp_version(void) { return "0.1.0"; }

const char* nnp_last_error(void) { return g_last_error.c_str(); }

const char* nnp_status_string(nnp_status s) {
  switch (s) {
    case NNP_OK: return "ok";
    case NNP_EINVAL: return "invalid argument";
    case NNP_ESPECIES: return "atomic number not in the species table";
    case NNP_EBOX: return "box length not larger than twice the cutoff";
    case NNP_ECAPACITY: return "capacity exceeded";
    case NNP_EHIP: return "HIP runtime error";
    case NNP_ESTATE: return "invalid call sequence";
    case NNP_ENONFINITE: return "non-finite position or energy";
  }
  return "unknown status";
}

nnp_status nnp_create(const nnp_config* cfg, uint64_t seed, const float* weights_host, nnp_precision prec,
                      nnp_model** out) {
  if (!cfg || !out) return set_error(NNP_EINVAL, "null argument");
  *out = nullptr;
  const int S = cfg->n_species;
  if (S < 1 || S > kMaxSpecies || !cfg->atomic_numbers_host)
    return set_error(NNP_EINVAL, "n_species must be 1..4 with an atomic number table");
  for (int s = 1; s < S; ++s)
    if (cfg->atomic_numbers_host[s] <= cfg->atomic_numbers_host[s - 1])
      return set_error(NNP_EINVAL, "atomic numbers must be strictly ascending");
  if (cfg->n_rad_shift != kRadShifts || cfg->n_ang_shift != kAngShifts || cfg->n_ang_sect != kAngSects ||
      !cfg->rad_shift_host || !cfg->ang_shift_host || !cfg->ang_sect_host)
    return set_error(NNP_EINVAL, "the descriptor needs 16 radial shifts, 8 angular shifts and 4 sections");
  if (!(cfg->rc_rad > 0.f) || !(cfg->rc_ang > 0.f) || cfg->rc_ang > cfg->rc_rad || !(cfg->eta_rad > 0.f) ||
      !(cfg->eta_ang > 0.f) || !(cfg->zeta > 0.f) || !(cfg->celu_alpha > 0.f))
    return set_error(NNP_EINVAL, "cutoffs, widths and exponents must be positive, rc_ang <= rc_rad");
  if (cfg->extra_inputs != 0 && cfg->extra_inputs != 1) return set_error(NNP_EINVAL, "extra_inputs must be 0 or 1");
  if (cfg->extra_inputs && !(cfg->mm_cutoff > 0.f)) return set_error(NNP_EINVAL, "mm_cutoff must be positive");
  if (cfg->n_members < 1) return set_error(NNP_EINVAL, "n_members must be >= 1");
  if (cfg->n_layers != 5 || !cfg->widths_host) return set_error(NNP_EINVAL, "networks have 5 widths (4 layers)");
  if (prec != NNP_FP32 && prec != NNP_BF16) return set_error(NNP_EINVAL, "unknown precision");
  const int D = descriptor_length(S);
  std::vector<int> w(cfg->widths_host, cfg->widths_host + 5);
  if (w[0] != D + cfg->extra_inputs || !(w[4] == 1 || (w[4] == 2 && cfg->extra_inputs == 1)))
    return set_error(NNP_EINVAL,
                     "widths[0] must equal the descriptor length plus extra_inputs; widths[4] = 1, or 2 (energy "
                     "and a predicted charge) with the MM potential channel");
  int kind = -1, stride = 0;
  if (w[1] == 160 && w[2] == 128 && w[3] == 96 && D == 128 && cfg->extra_inputs == 0) {
    kind = 0; stride = 128;
  } else if (w[1] == 256 && w[2] == 192 && w[3] == 160 && D == 384) {
    kind = cfg->extra_inputs ? 2 : 1;
    stride = cfg->extra_inputs ? 416 : 384;
  }
  if (kind < 0)
    return set_error(NNP_EINVAL,
                     "supported networks: 2 species 128-160-128-96-1, 4 species 384(+1)-256-192-160-1");

  nnp_model* m = new (std::nothrow) nnp_model();
  if (!m) return set_error(NNP_EINVAL, "out of host memory");
  (void)hipGetDevice(&m->device);
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) == hipSuccess && cus > 0)
      m->n_cu = cus;
  }
  m->prec = prec;
  m->S = S;
  m->P = S * (S + 1) / 2;
  m->D = D;
  m->extra = cfg->extra_inputs;
  m->charges = w[4] == 2;
  m->Din = D + cfg->extra_inputs;
  m->stride = stride;
  m->n_members = cfg->n_members;
  m->species.assign(cfg->atomic_numbers_host, cfg->atomic_numbers_host + S);
  m->widths = w;
  m->celu_alpha = cfg->celu_alpha;
  m->net_kind = kind;

  DescParams& p = m->dp;
  p.rc_rad = cfg->rc_rad;
  p.rc_ang = cfg->rc_ang;
  p.eta_rad = cfg->eta_rad;
  p.eta_ang = cfg->eta_ang;
  p.zeta = cfg->zeta;
  p.ang_pref = (float)std::pow(2.0, 1.0 - (double)cfg->zeta);
  for (int k = 0; k < kRadShifts; ++k) p.rad_shift[k] = cfg->rad_shift_host[k];
  for (int k = 0; k < kAngShifts; ++k) p.ang_shift[k] = cfg->ang_shift_host[k];
  for (int k = 0; k < kAngSects; ++k) {
    p.cos_sect[k] = (float)std::cos((double)cfg->ang_sect_host[k]);
    p.sin_sect[k] = (float)std::sin((double)cfg->ang_sect_host[k]);
  }
  {
    const double l2e = 1.4426950408889634;
    const double sr = std::sqrt((double)cfg->eta_rad * l2e), sa = std::sqrt((double)cfg->eta_ang * l2e);
    p.sq_eta_r = (float)sr;
    p.hq_eta_a = (float)(0.5 * sa);
    p.sq_pref = (float)std::pow(2.0, 0.5 * (1.0 - (double)cfg->zeta));
    for (int k = 0; k < kRadShifts; ++k) p.rad_shift_s[k] = (float)(sr * (double)cfg->rad_shift_host[k]);
    for (int k = 0; k < kAngShifts; ++k) p.ang_shift_s[k] = (float)(sa * (double)cfg->ang_shift_host[k]);
  }
  {
    const float pi = 3.14159265358979323846f;
    p.inv2rc = 0.5f / p.rc_rad;
    p.inv2rca = 0.5f / p.rc_ang;
    p.dfc_r = -0.5f * pi / p.rc_rad;
    p.dfc_a = -0.5f * pi / p.rc_ang;
    p.c1_rad = -2.f * p.eta_rad / p.sq_eta_r;
    p.c_sdr = -p.eta_ang / p.hq_eta_a;
  }
  p.mm_cutoff = cfg->mm_cutoff;
  p.ke = (float)cfg->ke_coulomb;
  p.S = S;
  p.P = m->P;
  p.D = D;
  p.stride = stride;
  p.extra = cfg->extra_inputs;
  int q = 0;
  for (int a = 0; a < S; ++a)
    for (int b = a; b < S; ++b) {
      p.pair_a[q] = a;
      p.pair_b[q] = b;
      p.class_of[a][b] = q;
      p.class_of[b][a] = q;
      ++q;
    }
  p.class_tab = 0;
  for (int a = 0; a < S; ++a)
    for (int b = 0; b < S; ++b) p.class_tab |= (uint64_t)p.class_of[a][b] << (4 * (4 * a + b));

  // weights
  size_t per_species = 0;
  for (int l = 0; l < 4; ++l) per_species += (size_t)w[l] * w[l + 1] + w[l + 1];
  const size_t total = per_species * S * m->n_members;
  if (weights_host) {
    m->w_host.assign(weights_host, weights_host + total);
  } else {
    draw_weights(seed, w, S, m->n_members, m->w_host);
  }
  std::vector<uint8_t> mat;
  std::vector<float> vec;
  pack_weights(*m, mat, vec, m->mat_per_species, m->vec_per_species);
  hipError_t e = hipMalloc(&m->d_wmat, mat.size());
  if (e == hipSuccess) e = hipMemcpy(m->d_wmat, mat.data(), mat.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = dalloc(&m->d_wvec, vec.size());
  if (e == hipSuccess) e = hipMemcpy(m->d_wvec, vec.data(), vec.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess && prec == NNP_BF16) {
    std::vector<uint16_t> rows;
    pack_rows_bf16(*m, rows, m->wrow_per_species);
    e = hipMalloc(&m->d_wrow, rows.size() * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemcpy(m->d_wrow, rows.data(), rows.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = dalloc(&m->d_status, 1);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMemset(m->d_status, 0, sizeof(int));
  if (e != hipSuccess) {
    nnp_destroy(m);
    return hip_error(e, "nnp_create");
  }
  {
    nnp_status st = noalloc_scratch_setup(m->device);
    if (st != NNP_OK) {
      nnp_destroy(m);
      return st;
    }
  }
  load_tuning(m);
  *out = m;
  return NNP_OK;
}

nnp_status nnp_reserve(nnp_model* m, int32_t max_atoms, int32_t max_systems, int32_t max_mm, int32_t max_rad_nbr,
                       int32_t max_ang_nbr) {
  if (!m) return set_error(NNP_EINVAL, "null model");
  if (max_atoms < 1 || max_systems < 1 || max_mm < 0 || max_rad_nbr < 0 || max_ang_nbr < 0)
    return set_error(NNP_EINVAL, "capacities must be positive");
  if (max_rad_nbr > 1024 || max_ang_nbr > 256)
    return set_error(NNP_EINVAL, "neighbour capacities are limited to 1024 (radial) and 256 (angular)");
  HIP_TRY(hipDeviceSynchronize(), "nnp_reserve");
  free_workspace(m);
  Workspace w = workspace_caps(*m, max_atoms, max_systems, max_mm, max_rad_nbr ? max_rad_nbr : 128,
                               max_ang_nbr ? max_ang_nbr : 64);
  const size_t bytes = carve_workspace(*m, w, nullptr);
  hipError_t e = hipMalloc(&m->d_ws_base, bytes);
  if (e == hipSuccess) {
    carve_workspace(*m, w, static_cast<char*>(m->d_ws_base));
    static_cast<Workspace&>(*m) = w;
    // the histogram starts from zero (every call leaves it cleared); descriptor
    // padding columns stay zero
    e = hipMemset(m->d_bin_count, 0, (size_t)m->max_bins * sizeof(int));
  }
  if (e == hipSuccess) e = hipMemset(m->d_x, 0, (size_t)max_atoms * m->stride * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->d_g, 0, (size_t)max_atoms * m->stride * sizeof(float));
  if (e == hipSuccess) {
    size_t stage = 3 * (size_t)max_atoms + 8;
    if (8 * (size_t)max_systems + 8 > stage) stage = 8 * (size_t)max_systems + 8;
    e = hipHostMalloc(reinterpret_cast<void**>(&m->h_stage), stage * sizeof(int), hipHostMallocDefault);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_workspace(m);
    return hip_error(e, "nnp_reserve");
  }
  m->reserved = true;
  return NNP_OK;
}

}  // extern "C"

namespace nnp {

// Box checks and the cell grid of a periodic call.
nnp_status setup_periodic(nnp_model* m, const float* box) {
  m->geo = Geometry{};
  Geometry& g = m->geo;
  g.periodic = 1;
  const float rc = m->dp.rc_rad;
  long long cells = 1;
  for (int k = 0; k < 3; ++k) {
    float L = box[k];
    if (!(std::isfinite(L)) || !(L > 2.f * rc))
      return set_error(NNP_EBOX, "box length " + std::to_string(L) + " must exceed twice the cutoff");
    if (m->extra && !(L > 2.f * m->dp.mm_cutoff))
      return set_error(NNP_EBOX, "box length must exceed twice the MM cutoff");
    g.box[k] = L;
    g.inv_box[k] = 1.0f / L;
    float q = std::floor(L / rc);
    g.nc[k] = q < 1.f ? 1 : (q > (float)kMaxCellsPerDim ? kMaxCellsPerDim : (int)q);
    cells *= g.nc[k];
  }
  // keep the grid within the reserved bins (larger cells stay correct)
  const long long cap = m->max_bins / m->S;
  while (cells > cap) {
    int k = 0;
    for (int d = 1; d < 3; ++d)
      if (g.nc[d] > g.nc[k]) k = d;
    g.nc[k] = g.nc[k] > 1 ? g.nc[k] / 2 : 1;
    cells = (long long)g.nc[0] * g.nc[1] * g.nc[2];
  }
  for (int k = 0; k < 3; ++k) {
    g.cell_scale[k] = (float)g.nc[k] * g.inv_box[k];
    g.cell_len[k] = g.box[k] / (float)g.nc[k];
  }
  g.n_bins = (int)cells;
  return NNP_OK;
}

// Stage timing: event pair (start, stop) of stage `st` in the current call.
struct StageTimer {
  nnp_model* m;
  hipStream_t s;
  bool on;
  StageTimer(nnp_model* mm, hipStream_t ss) : m(mm), s(ss), on(mm->prof_calls < mm->prof_max_calls) {}
  void mark(int stage, int which) {
    if (on) (void)hipEventRecord(m->prof_ev[((size_t)m->prof_calls * NNP_STAGE_COUNT + stage) * 2 + which], s);
  }
  void done() {
    if (on) ++m->prof_calls;
  }
};

#define STAGE(id, call, what)                          \
  do {                                                 \
    tm.mark(id, 0);                                    \
    hipError_t e_ = (call);                            \
    tm.mark(id, 1);                                    \
    if (e_ != hipSuccess) return hip_error(e_, what);  \
  } while (0)

nnp_status run_path(nnp_model* m, int n, const float* pos, int n_mm, const float* mm_pos, const float* mm_q,
                    double* energies, int n_sys, double* forces, double* mm_forces, int accumulate,
                    int assign_forces, int n_atoms, int n_pairs, const int* pairs, hipStream_t st) {
  m->last_n = n;
  StageTimer tm(m, st);
  STAGE(NNP_STAGE_CELLS, launch_cells(*m, pos, n, st), "cell list");
  if (pairs != nullptr || n_pairs > 0)
    STAGE(NNP_STAGE_NEIGHBOURS, launch_pair_lists(*m, n, n_atoms, n_pairs, pairs, st), "pair lists");
  else
    STAGE(NNP_STAGE_NEIGHBOURS, launch_neighbours(*m, n, st), "neighbours");
  STAGE(NNP_STAGE_DESCRIPTOR, launch_descriptor_fwd(*m, n, st), "descriptor");
  if (m->extra) STAGE(NNP_STAGE_MM, launch_mm_fwd(*m, n, n_mm, mm_pos, mm_q, st), "mm channel");
  STAGE(NNP_STAGE_NETWORK, launch_mlp(*m, n, st), "network");
  STAGE(NNP_STAGE_ADJOINT, launch_descriptor_bwd(*m, n, st), "descriptor adjoint");
  STAGE(NNP_STAGE_GATHER, launch_force_gather(*m, n, forces, assign_forces, energies, n_sys, accumulate, st),
        "force gather and energy");
  if (m->extra)
    STAGE(NNP_STAGE_MM_ADJOINT, launch_mm_bwd(*m, n, n_mm, mm_pos, mm_q, forces, mm_forces, st), "mm adjoint");
  tm.done();
  return NNP_OK;
}

}  // namespace nnp

extern "C" {

namespace {

// One system (periodic box or open), neighbour lists from the cell list or,
// with `pairs`, from the caller's pair list.
nnp_status compute_single(nnp_model* m, int32_t n_atoms, const float* pos, const int32_t* Z_host,
                          const float* box_host, int32_t n_nnp, const int32_t* nnp_idx_host, int32_t n_mm,
                          const float* mm_pos, const float* mm_q, double* energy, double* forces,
                          double* mm_forces, int32_t accumulate, int32_t n_pairs, const int32_t* pairs,
                          hipStream_t stream) {
  if (!m) return set_error(NNP_EINVAL, "null model");
  if (!m->reserved) return set_error(NNP_ESTATE, "nnp_reserve must be called first");
  if (n_atoms < 0 || n_nnp < 0 || n_nnp > n_atoms) return set_error(NNP_EINVAL, "bad atom counts");
  if (n_atoms > m->max_atoms)
    return set_error(NNP_ECAPACITY, "n_atoms exceeds the reserved capacity " + std::to_string(m->max_atoms));
  if (!energy || (n_atoms > 0 && (!pos || !forces))) return set_error(NNP_EINVAL, "null output or position array");
  if (m->extra) {
    if (n_mm < 0 || (n_mm > 0 && (!mm_pos || !mm_q)))
      return set_error(NNP_EINVAL, "this model needs MM positions and charges");
    if (n_mm > m->max_mm) return set_error(NNP_ECAPACITY, "n_mm exceeds the reserved capacity");
  } else if (n_mm != 0) {
    return set_error(NNP_EINVAL, "MM charges given to a model without the MM input channel");
  }
  if (accumulate != 0 && accumulate != 1) return set_error(NNP_EINVAL, "accumulate must be 0 or 1");

  const bool pair_mode = pairs != nullptr || n_pairs != 0;
  if (pair_mode) {
    if (n_pairs < 0 || (n_pairs > 0 && !pairs)) return set_error(NNP_EINVAL, "bad pair list");
    if (m->max_rad > kPairRowMax)
      return set_error(NNP_EINVAL, "pair lists need max_rad_nbr <= " + std::to_string(kPairRowMax));
  }

  // topology (index group plus link atoms)
  const int n_links = m->n_links_dev;
  if (n_nnp + n_links > m->max_atoms)
    return set_error(NNP_ECAPACITY, "NNP atoms plus link atoms exceed the reserved capacity");
  if (Z_host) {
    bool same = m->topo_mode == 0 && m->topo_n_atoms == n_atoms && m->n_nnp == n_nnp &&
                m->topo_link_version == m->link_version &&
                std::memcmp(m->topo_Z.data(), Z_host, sizeof(int) * (size_t)n_atoms) == 0;
    if (same) {
      if (nnp_idx_host)
        same = m->topo_idx.size() == (size_t)n_nnp &&
               std::memcmp(m->topo_idx.data(), nnp_idx_host, sizeof(int) * (size_t)n_nnp) == 0;
      else
        same = m->topo_idx.empty();
    }
    if (!same) {
      if (!nnp_idx_host && n_nnp != n_atoms) return set_error(NNP_EINVAL, "nnp_idx is NULL but n_nnp != n_atoms");
      const int n_loc = n_nnp + n_links;
      std::vector<int> idx(n_loc), sig(n_loc);
      std::vector<char> seen(n_atoms, 0);
      for (int t = 0; t < n_nnp; ++t) {
        int a = nnp_idx_host ? nnp_idx_host[t] : t;
        if (a < 0 || a >= n_atoms || seen[a]) return set_error(NNP_EINVAL, "index group entries must be distinct and in range");
        seen[a] = 1;
        idx[t] = a;
        nnp_status s = species_of(m, Z_host[a], &sig[t]);
        if (s != NNP_OK) return s;
      }
      for (int l = 0; l < n_links; ++l) {
        const int a = m->link_ml[l], b = m->link_mm[l];
        if (a < 0 || a >= n_atoms || b < 0 || b >= n_atoms || !seen[a] || seen[b])
          return set_error(NNP_EINVAL, "each link needs its ML atom inside and its MM atom outside the index group");
        idx[n_nnp + l] = -1 - l;
        sig[n_nnp + l] = m->link_sigma;
      }
      nnp_status s;
      if ((s = upload_ints(m, m->d_idx, idx.data(), n_loc, stream)) != NNP_OK) return s;
      if ((s = upload_ints(m, m->d_sigma, sig.data(), n_loc, stream)) != NNP_OK) return s;
      std::vector<int> zeros(n_loc, 0);  // an open single system is system 0
      if ((s = upload_ints(m, m->d_sys, zeros.data(), n_loc, stream)) != NNP_OK) return s;
      std::vector<int> loc(n_atoms, -1);  // system atom -> NNP-local index (pair lists)
      for (int t = 0; t < n_nnp; ++t) loc[idx[t]] = t;
      if (n_atoms > 0 && (s = upload_ints(m, m->d_loc, loc.data(), n_atoms, stream)) != NNP_OK) return s;
      const int off[2] = {0, n_loc};
      if ((s = upload_ints(m, m->d_sys_off, off, 2, stream)) != NNP_OK) return s;
      m->topo_mode = 0;
      m->topo_n_atoms = n_atoms;
      m->n_nnp = n_nnp;
      m->topo_link_version = m->link_version;
      m->topo_Z.assign(Z_host, Z_host + n_atoms);
      if (nnp_idx_host) m->topo_idx.assign(nnp_idx_host, nnp_idx_host + n_nnp);
      else m->topo_idx.clear();
    }
  } else if (m->topo_mode != 0 || m->topo_n_atoms != n_atoms || m->n_nnp != n_nnp ||
             m->topo_link_version != m->link_version) {
    return set_error(NNP_ESTATE, "Z_host is NULL but no matching topology was given before");
  }
  const int n_loc = n_nnp + n_links;

  // geometry
  if (box_host) {
    nnp_status s = setup_periodic(m, box_host);
    if (s != NNP_OK) return s;
  } else {
    m->geo = Geometry{};
    m->geo.periodic = 0;
    m->geo.n_bins = 1;
    m->geo.nc[0] = m->geo.nc[1] = m->geo.nc[2] = 1;
  }
  m->last_n = n_loc;
  auto launch = [=](hipStream_t s) -> nnp_status {
    hipError_t e;
    // with every atom in the index group the gather overwrites each force row
    const int assign = !accumulate && n_nnp == n_atoms;
    if (!accumulate) {
      if (!assign && (e = launch_fill_f64(forces, 3 * (int64_t)n_atoms, s)) != hipSuccess)
        return hip_error(e, "fill");
      if (mm_forces && (e = launch_fill_f64(mm_forces, 3 * (int64_t)n_mm, s)) != hipSuccess)
        return hip_error(e, "fill");
    }
    if (n_links > 0 && (e = launch_fill_f64(m->d_link_F, 3 * (int64_t)n_links, s)) != hipSuccess)
      return hip_error(e, "fill");
    nnp_status st =
        run_path(m, n_loc, pos, n_mm, mm_pos, mm_q, energy, 1, forces, mm_forces, accumulate, assign, n_atoms, n_pairs,
                 pairs, s);
    if (st != NNP_OK) return st;
    if (n_links > 0 && (e = launch_link_redistribute(*m, pos, forces, s)) != hipSuccess)
      return hip_error(e, "link atoms");
    return NNP_OK;
  };
  const int mode = pair_mode ? 2 : 0;
  const int lv = m->link_version;
  return dispatch(m, make_key(mode, pos, energy, forces, mm_forces, mm_pos, mm_q, n_atoms, n_nnp, n_mm, accumulate,
                              lv, m->geo, n_pairs, pairs),
                  stream, launch);
}

}  // namespace

nnp_status nnp_compute(nnp_model* m, int32_t n_atoms, const float* pos, const int32_t* Z_host, const float* box_host,
                       int32_t n_nnp, const int32_t* nnp_idx_host, int32_t n_mm, const float* mm_pos,
                       const float* mm_q, double* energy, double* forces, double* mm_forces, int32_t accumulate,
                       hipStream_t stream) {
  return compute_single(m, n_atoms, pos, Z_host, box_host, n_nnp, nnp_idx_host, n_mm, mm_pos, mm_q, energy, forces,
                        mm_forces, accumulate, 0, nullptr, stream);
}

nnp_status nnp_compute_pairs(nnp_model* m, int32_t n_atoms, const float* pos, const int32_t* Z_host,
                             const float* box_host, int32_t n_nnp, const int32_t* nnp_idx_host, int32_t n_pairs,
                             const int32_t* pairs, int32_t n_mm, const float* mm_pos, const float* mm_q,
                             double* energy, double* forces, double* mm_forces, int32_t accumulate,
                             hipStream_t stream) {
  if (n_pairs > 0 && !pairs) return set_error(NNP_EINVAL, "null pair list");
  if (n_pairs < 0) return set_error(NNP_EINVAL, "bad pair count");
  // an empty list still selects the pair path (every NNP atom then has no neighbour)
  static const int32_t kNone[2] = {0, 0};
  return compute_single(m, n_atoms, pos, Z_host, box_host, n_nnp, nnp_idx_host, n_mm, mm_pos, mm_q, energy, forces,
                        mm_forces, accumulate, n_pairs, pairs ? pairs : kNone, stream);
}

nnp_status nnp_compute_batch(nnp_model* m, int32_t n_sys, const int32_t* atom_offsets_host, const float* pos,
                             const int32_t* Z_host, const float* boxes_host, double* energies, double* forces,
                             hipStream_t stream) {
  if (!m) return set_error(NNP_EINVAL, "null model");
  if (!m->reserved) return set_error(NNP_ESTATE, "nnp_reserve must be called first");
  if (m->extra) return set_error(NNP_EINVAL, "batched calls do not take MM charges");
  if (n_sys < 1 || !atom_offsets_host) return set_error(NNP_EINVAL, "need at least one system and its offsets");
  if (n_sys > m->max_sys) return set_error(NNP_ECAPACITY, "n_sys exceeds the reserved capacity");
  if (atom_offsets_host[0] != 0) return set_error(NNP_EINVAL, "atom_offsets[0] must be 0");
  for (int s = 0; s < n_sys; ++s)
    if (atom_offsets_host[s + 1] < atom_offsets_host[s]) return set_error(NNP_EINVAL, "offsets must be non-decreasing");
  const int n = atom_offsets_host[n_sys];
  if (n > m->max_atoms) return set_error(NNP_ECAPACITY, "total atoms exceed the reserved capacity");
  if (!energies || (n > 0 && (!pos || !forces))) return set_error(NNP_EINVAL, "null output or position array");

  // per-system boxes: (L, 1/L) in FP32 per system, zeros for an open system
  std::vector<float> boxes;
  if (boxes_host) {
    boxes.assign(8 * (size_t)n_sys, 0.f);
    const float rc = m->dp.rc_rad;
    for (int s = 0; s < n_sys; ++s) {
      const float* b = boxes_host + 3 * (size_t)s;
      const bool open = b[0] == 0.f && b[1] == 0.f && b[2] == 0.f;
      if (open) continue;
      for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(b[k]) || !(b[k] > 2.f * rc))
          return set_error(NNP_EBOX, "system " + std::to_string(s) + ": box length " + std::to_string(b[k]) +
                                         " must exceed twice the cutoff (or the whole row be 0 for an open system)");
        boxes[8 * (size_t)s + k] = b[k];
        boxes[8 * (size_t)s + 4 + k] = 1.0f / b[k];
      }
    }
  }

  if (Z_host) {
    bool same = m->topo_mode == 1 && m->topo_n_atoms == n && (int)m->topo_offsets.size() == n_sys + 1 &&
                std::memcmp(m->topo_offsets.data(), atom_offsets_host, sizeof(int) * (size_t)(n_sys + 1)) == 0 &&
                std::memcmp(m->topo_Z.data(), Z_host, sizeof(int) * (size_t)n) == 0;
    if (!same) {
      std::vector<int> idx(n), sig(n), sys(n);
      for (int s = 0; s < n_sys; ++s)
        for (int a = atom_offsets_host[s]; a < atom_offsets_host[s + 1]; ++a) sys[a] = s;
      for (int a = 0; a < n; ++a) {
        idx[a] = a;
        nnp_status st = species_of(m, Z_host[a], &sig[a]);
        if (st != NNP_OK) return st;
      }
      nnp_status st;
      if ((st = upload_ints(m, m->d_idx, idx.data(), n, stream)) != NNP_OK) return st;
      if ((st = upload_ints(m, m->d_sigma, sig.data(), n, stream)) != NNP_OK) return st;
      if ((st = upload_ints(m, m->d_sys, sys.data(), n, stream)) != NNP_OK) return st;
      if ((st = upload_ints(m, m->d_sys_off, atom_offsets_host, n_sys + 1, stream)) != NNP_OK) return st;
      m->topo_mode = 1;
      m->topo_n_atoms = n;
      m->n_nnp = n;
      m->topo_Z.assign(Z_host, Z_host + n);
      m->topo_offsets.assign(atom_offsets_host, atom_offsets_host + n_sys + 1);
      m->topo_idx.clear();
      m->topo_boxes.clear();
    }
  } else if (m->topo_mode != 1 || m->topo_n_atoms != n || (int)m->topo_offsets.size() != n_sys + 1) {
    return set_error(NNP_ESTATE, "Z_host is NULL but no matching batched topology was given before");
  }
  // the boxes live in device memory, so a captured graph stays valid when they change
  if (boxes_host && boxes != m->topo_boxes) {
    nnp_status st = upload_words(m, m->d_sys_box, boxes.data(), 8 * n_sys, stream);
    if (st != NNP_OK) return st;
    m->topo_boxes = boxes;
  }
  m->geo = Geometry{};
  m->geo.periodic = 0;
  m->geo.n_bins = n_sys;
  m->geo.nc[0] = m->geo.nc[1] = m->geo.nc[2] = 1;
  m->geo.sys_box = boxes_host ? m->d_sys_box : nullptr;
  m->geo.sbin = m->d_sbin;
  if (m->S * n_sys > m->max_bins) return set_error(NNP_ECAPACITY, "too many systems for the reserved bins");
  m->last_n = n;
  auto launch = [=](hipStream_t s) -> nnp_status {
    // every atom of a batched call is an NNP atom: the gather overwrites each force row
    return run_path(m, n, pos, 0, nullptr, nullptr, energies, n_sys, forces, nullptr, 0, 1, n, 0, nullptr, s);
  };
  const int mode = 1;
  return dispatch(m, make_key(mode, pos, energies, forces, n, n_sys, m->geo), stream, launch);
}

nnp_status nnp_get_status(nnp_model* m, hipStream_t stream) {
  if (!m || !m->d_status) return set_error(NNP_EINVAL, "null model");
  HIP_TRY(hipStreamSynchronize(stream), "nnp_get_status");
  int h = 0;
  HIP_TRY(hipMemcpy(&h, m->d_status, sizeof(int), hipMemcpyDeviceToHost), "nnp_get_status");
  HIP_TRY(hipMemset(m->d_status, 0, sizeof(int)), "nnp_get_status");
  if (h & kStatusCapacity) return set_error(NNP_ECAPACITY, "a neighbour list overflowed its capacity");
  if (h & kStatusNonFinite) return set_error(NNP_ENONFINITE, "non-finite position or energy");
  if (h & kStatusInput) return set_error(NNP_EINVAL, "the pair list held an out-of-range, self or repeated pair");
  return NNP_OK;
}

nnp_status nnp_read_buffer(nnp_model* m, nnp_buffer which, void* dst_host, size_t capacity_bytes, int64_t* elems,
                           int32_t* row_stride, hipStream_t stream) {
  if (!m || !elems || !row_stride) return set_error(NNP_EINVAL, "null argument");
  if (!m->reserved) return set_error(NNP_ESTATE, "nothing computed yet");
  HIP_TRY(hipStreamSynchronize(stream), "nnp_read_buffer");
  const int n = m->last_n;
  const void* src = nullptr;
  size_t esz = 4;
  int64_t count = 0;
  int32_t stride = 1;
  std::vector<int> tmp;
  switch (which) {
    case NNP_BUF_PERM: src = m->d_perm; count = n; break;
    case NNP_BUF_KEY: src = m->d_key; count = n; break;
    case NNP_BUF_ORDER: src = m->d_order; count = n; break;
    case NNP_BUF_BIN_START: src = m->d_bin_start; count = (int64_t)m->S * m->geo.n_bins + 1; break;
    case NNP_BUF_NBR_RAD: src = m->d_nbr_rad; count = (int64_t)n * m->max_rad; stride = m->max_rad; break;
    case NNP_BUF_NBR_ANG: src = m->d_nbr_ang; count = (int64_t)n * m->max_ang; stride = m->max_ang; break;
    case NNP_BUF_DESCRIPTOR: src = m->d_x; count = (int64_t)n * m->stride; stride = m->stride; break;
    case NNP_BUF_ATOM_ENERGY: src = m->d_e; count = n; break;
    case NNP_BUF_CHARGE:
      if (!m->charges) return set_error(NNP_EINVAL, "the model has no charge output");
      src = m->d_q;
      count = n;
      break;
    case NNP_BUF_DEDX: src = m->d_g; count = (int64_t)n * m->stride; stride = m->stride; break;
    case NNP_BUF_NBR_COUNT: {
      std::vector<int> ro((size_t)n * (m->S + 1)), ao((size_t)n * (m->S + 1));
      if (n > 0) {
        HIP_TRY(hipMemcpy(ro.data(), m->d_rad_off, ro.size() * 4, hipMemcpyDeviceToHost), "read");
        HIP_TRY(hipMemcpy(ao.data(), m->d_ang_off, ao.size() * 4, hipMemcpyDeviceToHost), "read");
      }
      tmp.resize((size_t)2 * n);
      for (int i = 0; i < n; ++i) {
        tmp[2 * i] = ro[(size_t)i * (m->S + 1) + m->S];
        tmp[2 * i + 1] = ao[(size_t)i * (m->S + 1) + m->S];
      }
      count = 2 * (int64_t)n;
      stride = 2;
      break;
    }
    case NNP_BUF_GRID: {
      tmp = {m->geo.n_bins, m->geo.nc[0], m->geo.nc[1], m->geo.nc[2]};
      count = 4;
      break;
    }
    case NNP_BUF_GRAPH: {
      auto clamp = [](int64_t v) { return (int)(v > 0x7fffffff ? 0x7fffffff : v); };
      tmp = {clamp(m->graph_builds), clamp(m->graph_updates), clamp(m->graph_replays)};
      count = 3;
      break;
    }
    default: return set_error(NNP_EINVAL, "unknown buffer");
  }
  *elems = count;
  *row_stride = stride;
  size_t bytes = (size_t)count * esz;
  if (bytes > capacity_bytes) bytes = capacity_bytes;
  if (bytes == 0) return NNP_OK;
  if (!dst_host) return set_error(NNP_EINVAL, "null destination");
  if (!tmp.empty() || which == NNP_BUF_NBR_COUNT || which == NNP_BUF_GRID || which == NNP_BUF_GRAPH) {
    std::memcpy(dst_host, tmp.data(), bytes);
  } else {
    HIP_TRY(hipMemcpy(dst_host, src, bytes, hipMemcpyDeviceToHost), "nnp_read_buffer");
  }
  return NNP_OK;
}

nnp_status nnp_autotune(nnp_model* m, int32_t reps, int32_t* chosen, hipStream_t stream) {
  if (!m || reps < 1 || reps > 256) return set_error(NNP_EINVAL, "bad argument");
  if (!m->reserved || m->last_n <= 0) return set_error(NNP_ESTATE, "nnp_autotune needs a previous compute call");
  HIP_TRY(hipStreamSynchronize(stream), "nnp_autotune");
  drop_graph(m);
  const int n = m->last_n;
  // Each candidate is timed in context: the stages after the cell list run in
  // their usual order on the previous call's workspace (positions already
  // sorted; nothing of the caller's is read or written), with events around
  // the stage being tuned only.
  std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  auto destroy = [&]() {
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
  };
  if (e != hipSuccess) {
    destroy();
    return hip_error(e, "nnp_autotune");
  }
  auto pass = [&](int stage, hipEvent_t e0, hipEvent_t e1) -> hipError_t {
    hipError_t r = hipSuccess;
    auto timed = [&](int st_id, auto&& launch) {
      if (r != hipSuccess) return;
      if (st_id == stage && e0) r = hipEventRecord(e0, stream);
      if (r == hipSuccess) r = launch();
      if (r == hipSuccess && st_id == stage && e1) r = hipEventRecord(e1, stream);
    };
    timed(kTuneNeighbours, [&] { return launch_neighbours(*m, n, stream); });
    timed(kTuneDescriptor, [&] { return launch_descriptor_fwd(*m, n, stream); });
    timed(kTuneNetwork, [&] { return launch_mlp(*m, n, stream); });
    timed(kTuneAdjoint, [&] { return launch_descriptor_bwd(*m, n, stream); });
    return r;
  };
  auto time_stage = [&](int stage, int v, float* ms) -> nnp_status {
    m->force_variant[stage] = v;
    hipError_t r = pass(stage, nullptr, nullptr);   // warm-up
    for (int k = 0; k < reps && r == hipSuccess; ++k) r = pass(stage, ev[2 * k], ev[2 * k + 1]);
    if (r == hipSuccess) r = hipStreamSynchronize(stream);
    *ms = 0.f;
    for (int k = 0; k < reps && r == hipSuccess; ++k) {
      float t = 0.f;
      r = hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]);
      *ms += t;
    }
    m->force_variant[stage] = -1;
    return r == hipSuccess ? NNP_OK : hip_error(r, "nnp_autotune");
  };
  const int stages[4] = {kTuneNetwork, kTuneDescriptor, kTuneAdjoint, kTuneNeighbours};
  nnp_status status = NNP_OK;
  for (int st : stages) {
    if (m->pinned[st] >= 0) continue;   // a pinned stage keeps its variant
    int nv = st == kTuneNeighbours && m->geo.n_bins < 2 ? 1 : kStageVariants[st];
    int best = 0;
    float best_ms = 0.f;
    for (int v = 0; v < nv && status == NNP_OK; ++v) {
      float ms = 0.f;
      status = time_stage(st, v, &ms);
      if (status == NNP_OK && (v == 0 || ms < best_ms)) {
        best_ms = ms;
        best = v;
      }
    }
    if (status != NNP_OK) break;
    m->tuned[{st, size_bucket(n)}] = best;
  }
  destroy();
  if (status != NNP_OK) return status;
  save_tuning(m);
  return chosen ? nnp_get_variants(m, chosen) : NNP_OK;
}

nnp_status nnp_get_variants(nnp_model* m, int32_t* chosen) {
  if (!m || !chosen) return set_error(NNP_EINVAL, "bad argument");
  if (!m->reserved || m->last_n <= 0) return set_error(NNP_ESTATE, "nnp_get_variants needs a previous compute call");
  chosen[kTuneNeighbours] = neighbour_variant(*m, m->last_n);
  chosen[kTuneDescriptor] = descriptor_variant(*m, m->last_n);
  chosen[kTuneNetwork] = mlp_variant(*m, m->last_n);
  chosen[kTuneAdjoint] = adjoint_variant(*m, m->last_n);
  return NNP_OK;
}

nnp_status nnp_set_links(nnp_model* m, int32_t n_links, const int32_t* ml_idx_host, const int32_t* mm_idx_host,
                         float distance, int32_t link_Z) {
  if (!m || n_links < 0) return set_error(NNP_EINVAL, "bad argument");
  if (n_links > 0 && (!ml_idx_host || !mm_idx_host)) return set_error(NNP_EINVAL, "null link index arrays");
  if (n_links > 0 && !(distance > 0.f)) return set_error(NNP_EINVAL, "link distance must be positive");
  int sig = 0;
  if (n_links > 0) {
    nnp_status s = species_of(m, link_Z, &sig);
    if (s != NNP_OK) return s;
  }
  HIP_TRY(hipDeviceSynchronize(), "nnp_set_links");
  drop_graph(m);
  dfree(m->d_link_ml);
  dfree(m->d_link_mm);
  dfree(m->d_link_F);
  m->link_ml.assign(ml_idx_host, ml_idx_host + n_links);
  m->link_mm.assign(mm_idx_host, mm_idx_host + n_links);
  m->link_d = distance;
  m->link_Z = link_Z;
  m->link_sigma = sig;
  m->n_links_dev = n_links;
  ++m->link_version;
  if (n_links > 0) {
    HIP_TRY(dalloc(&m->d_link_ml, (size_t)n_links), "nnp_set_links");
    HIP_TRY(dalloc(&m->d_link_mm, (size_t)n_links), "nnp_set_links");
    HIP_TRY(dalloc(&m->d_link_F, 3 * (size_t)n_links), "nnp_set_links");
    HIP_TRY(hipMemcpy(m->d_link_ml, ml_idx_host, sizeof(int) * (size_t)n_links, hipMemcpyHostToDevice), "nnp_set_links");
    HIP_TRY(hipMemcpy(m->d_link_mm, mm_idx_host, sizeof(int) * (size_t)n_links, hipMemcpyHostToDevice), "nnp_set_links");
  }
  return NNP_OK;
}

nnp_status nnp_set_graph(nnp_model* m, int32_t enable) {
  if (!m) return set_error(NNP_EINVAL, "null model");
  m->graph_enabled = enable != 0;
  if (!m->graph_enabled) drop_graph(m);
  return NNP_OK;
}

nnp_status nnp_me_coupling(int32_t n_ml, const float* ml_pos, const float* ml_param, int32_t n_mm,
                           const float* mm_pos, const float* mm_param, const float* box_host, float cutoff,
                           float ke, double* energy, double* ml_forces, double* mm_forces, int32_t accumulate,
                           hipStream_t stream) {
  if (n_ml < 0 || n_mm < 0) return set_error(NNP_EINVAL, "bad atom counts");
  if (!energy || (n_ml > 0 && (!ml_pos || !ml_param || !ml_forces)) ||
      (n_mm > 0 && (!mm_pos || !mm_param || !mm_forces)))
    return set_error(NNP_EINVAL, "null array");
  if (accumulate != 0 && accumulate != 1) return set_error(NNP_EINVAL, "accumulate must be 0 or 1");
  if (!(cutoff >= 0.f) || !std::isfinite(cutoff) || !std::isfinite(ke))
    return set_error(NNP_EINVAL, "cutoff must be finite and >= 0");
  Geometry g{};
  if (box_host) {
    if (!(cutoff > 0.f)) return set_error(NNP_EBOX, "a periodic box needs a cutoff");
    for (int k = 0; k < 3; ++k) {
      if (!(box_host[k] > 2.f * cutoff) || !std::isfinite(box_host[k]))
        return set_error(NNP_EBOX, "every box length must exceed twice the cutoff");
      g.box[k] = box_host[k];
      g.inv_box[k] = 1.f / box_host[k];
    }
    g.periodic = 1;
  }
  if (n_ml == 0 && n_mm == 0 && accumulate) return NNP_OK;
  hipError_t e = launch_me_pairs(n_ml, ml_pos, ml_param, n_mm, mm_pos, mm_param, g, cutoff, ke, energy, ml_forces,
                                 mm_forces, accumulate, stream);
  return e == hipSuccess ? NNP_OK : hip_error(e, "nnp_me_coupling");
}

nnp_status nnp_set_variant(nnp_model* m, int32_t stage, int32_t variant) {
  if (!m) return set_error(NNP_EINVAL, "null model");
  if (stage < 0 || stage >= kTuneStages) return set_error(NNP_EINVAL, "unknown stage");
  if (variant < -1 || variant >= kStageVariants[stage]) return set_error(NNP_EINVAL, "unknown variant");
  HIP_TRY(hipDeviceSynchronize(), "nnp_set_variant");
  drop_graph(m);
  m->pinned[stage] = variant;
  return NNP_OK;
}

nnp_status nnp_profile_enable(nnp_model* m, int32_t max_calls) {
  if (!m || max_calls < 0) return set_error(NNP_EINVAL, "bad argument");
  HIP_TRY(hipDeviceSynchronize(), "nnp_profile_enable");
  for (hipEvent_t e : m->prof_ev) (void)hipEventDestroy(e);
  m->prof_ev.clear();
  m->prof_calls = 0;
  m->prof_max_calls = 0;
  if (max_calls == 0) return NNP_OK;
  m->prof_ev.resize((size_t)max_calls * NNP_STAGE_COUNT * 2, nullptr);
  for (auto& e : m->prof_ev) HIP_TRY(hipEventCreate(&e), "nnp_profile_enable");
  m->prof_max_calls = max_calls;
  return NNP_OK;
}

nnp_status nnp_profile_read(nnp_model* m, double* ms_total, int64_t* calls, hipStream_t stream) {
  if (!m || !ms_total || !calls) return set_error(NNP_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(stream), "nnp_profile_read");
  for (int st = 0; st < NNP_STAGE_COUNT; ++st) ms_total[st] = 0.0;
  for (int c = 0; c < m->prof_calls; ++c)
    for (int st = 0; st < NNP_STAGE_COUNT; ++st) {
      hipEvent_t a = m->prof_ev[((size_t)c * NNP_STAGE_COUNT + st) * 2];
      hipEvent_t b = m->prof_ev[((size_t)c * NNP_STAGE_COUNT + st) * 2 + 1];
      float ms = 0.f;
      // stages a call skipped have no recorded events: hipEventElapsedTime fails, count 0
      if (hipEventQuery(a) == hipSuccess && hipEventQuery(b) == hipSuccess &&
          hipEventElapsedTime(&ms, a, b) == hipSuccess)
        ms_total[st] += ms;
    }
  *calls = m->prof_calls;
  (void)hipGetLastError();
  return NNP_OK;
}

void nnp_destroy(nnp_model* m) {
  if (!m) return;
  drop_graph(m);
  dfree(m->d_link_ml);
  dfree(m->d_link_mm);
  dfree(m->d_link_F);
  if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
  m->cap_stream = nullptr;
  for (hipEvent_t e : m->prof_ev) (void)hipEventDestroy(e);
  m->prof_ev.clear();
  (void)hipDeviceSynchronize();
  free_workspace(m);
  if (m->d_wmat) (void)hipFree(m->d_wmat);
  if (m->d_wrow) (void)hipFree(m->d_wrow);
  dfree(m->d_wvec);
  dfree(m->d_status);
  delete m;
}

}  // extern "C"
