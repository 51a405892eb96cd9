// The entry point that allocates nothing: nnp_compute's path for one system
// whose atoms are all NNP atoms, with the per-call workspace carved out of a
// static device array instead of the allocation nnp_reserve makes.  For
// callers that cannot allocate device memory at all.
//
// The array is a file-scope device variable of fixed size.  Its device
// address is looked up once per device (hipGetSymbolAddress, from nnp_create
// with that device current) and only that address is used on the host side;
// the host-side name of the array is a stand-in and never reaches a kernel.
// Every call on a device shares that device's array: calls that overlap on
// one device (two streams, two threads) race on it.  Nothing of a previous
// call is relied on: what must start at zero (the bin histogram) is cleared
// by this call's first kernel.
#include <mutex>

#include "nnp_internal.h"

namespace nnp {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

constexpr int kBlock = 256;

struct SpeciesTable {
  int z[kMaxSpecies];
  int S;
};

// Topology of an all-NNP single system from the uploaded atomic numbers (the
// host has already checked them against the table), and a cleared histogram.
__global__ __launch_bounds__(kBlock) void k_noalloc_setup(const int* __restrict__ Z, int n, SpeciesTable tab,
                                                          int* __restrict__ idx, int* __restrict__ sigma,
                                                          int* __restrict__ sys, int* __restrict__ sys_off,
                                                          int* __restrict__ bin_count, int n_keys) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    const int z = Z[t];
    int s = 0;
    for (int k = 1; k < tab.S; ++k)
      if (tab.z[k] == z) s = k;
    idx[t] = t;
    sigma[t] = s;
    sys[t] = 0;
  }
  if (t < n_keys) bin_count[t] = 0;
  if (t == 0) {
    sys_off[0] = 0;
    sys_off[1] = n;
  }
}

// The saved per-call state of the model, put back when the call returns.
struct Restore {
  nnp_model* m;
  Workspace ws;
  Geometry geo;
  int last_n;
  explicit Restore(nnp_model* mm) : m(mm), ws(*mm), geo(mm->geo), last_n(mm->last_n) {}
  ~Restore() {
    static_cast<Workspace&>(*m) = ws;
    m->geo = geo;
    m->last_n = last_n;
  }
};

}  // namespace

nnp_status noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return set_error(NNP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return NNP_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) return hip_error(e, "device address of the static workspace");
  g_scratch_ptr[device] = p;
  return NNP_OK;
}

}  // namespace nnp

using namespace nnp;

extern "C" nnp_status nnp_compute_noalloc(nnp_model* m, int32_t n_atoms, const float* pos, const int32_t* Z_host,
                                          const float* box_host, double* energy, double* forces,
                                          hipStream_t stream) {
  if (!m) return set_error(NNP_EINVAL, "null model");
  if (m->extra) return set_error(NNP_EINVAL, "models with the MM input channel need nnp_compute");
  if (m->n_links_dev > 0) return set_error(NNP_ESTATE, "link atoms are not supported by nnp_compute_noalloc");
  if (n_atoms < 1 || !pos || !Z_host || !energy || !forces)
    return set_error(NNP_EINVAL, "need at least one atom, positions, atomic numbers and outputs");
  for (int a = 0; a < n_atoms; ++a) {
    bool known = false;
    for (int s = 0; s < m->S; ++s) known = known || m->species[s] == Z_host[a];
    if (!known)
      return set_error(NNP_ESPECIES, "atomic number " + std::to_string(Z_host[a]) + " is not in the species table");
  }
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = m->device >= 0 && m->device < kMaxDevices ? g_scratch_ptr[m->device] : nullptr;
  }
  if (!base) return set_error(NNP_ESTATE, "the static workspace of this device was not set up");

  Workspace w = workspace_caps(*m, n_atoms, 1, 0, 128, 64);
  const size_t need = carve_workspace(*m, w, nullptr);
  if (need > kNoallocScratchBytes)
    return set_error(NNP_ECAPACITY, std::to_string(n_atoms) + " atoms need " + std::to_string(need) +
                                        " bytes of workspace; the static array holds " +
                                        std::to_string(kNoallocScratchBytes));
  carve_workspace(*m, w, static_cast<char*>(base));

  Restore restore(m);
  static_cast<Workspace&>(*m) = w;
  if (box_host) {
    nnp_status s = setup_periodic(m, box_host);
    if (s != NNP_OK) return s;
  } else {
    m->geo = Geometry{};
    m->geo.periodic = 0;
    m->geo.n_bins = 1;
    m->geo.nc[0] = m->geo.nc[1] = m->geo.nc[2] = 1;
  }
  m->last_n = n_atoms;

  // atomic numbers go to the scatter buffer, which the cell list overwrites later
  hipError_t e = hipMemcpyAsync(m->d_tmp, Z_host, sizeof(int) * (size_t)n_atoms, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_error(e, "atomic numbers");
  SpeciesTable tab{};
  tab.S = m->S;
  for (int s = 0; s < m->S; ++s) tab.z[s] = m->species[s];
  const int n_keys = m->S * m->geo.n_bins;
  const int cover = n_atoms > n_keys ? n_atoms : n_keys;
  hipLaunchKernelGGL(k_noalloc_setup, dim3((unsigned)((cover + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream,
                     m->d_tmp, n_atoms, tab, m->d_idx, m->d_sigma, m->d_sys, m->d_sys_off, m->d_bin_count, n_keys);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "topology");
  // all atoms are NNP atoms and the outputs are overwritten: the gather assigns every force row
  return run_path(m, n_atoms, pos, 0, nullptr, nullptr, energy, 1, forces, nullptr, 0, 1, n_atoms, 0, nullptr,
                  stream);
}
