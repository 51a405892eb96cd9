/*
 * nnp.h -- C ABI of an MI355X (gfx950) library that evaluates a descriptor-based
 * neural network potential (NNP) and its forces, for the ML atoms of a
 * molecular-dynamics system, on a caller's HIP stream.
 *
 * The operation is the per-step ML/MM force contract of Muellender, Hess and
 * Lindahl, "Enabling Biomolecular Simulations with Neural Network Potentials in
 * GROMACS" (arXiv 2604.21441):
 *   - the NNP supplies the energy E_ML of an index group of atoms (Theory,
 *     eq. 1) and the forces F_i = -grad_i E_ML on those atoms (eq. 2);
 *   - its inputs are atomic numbers, positions, the box and periodicity, the
 *     index group, and optionally MM positions and charges (Methods, "The
 *     nnpot Interface"); with MM charges the model may also put forces on MM
 *     atoms (same passage, electrostatic embedding).
 * The model is an ANI-family network (the family the paper runs and
 * benchmarks): radial and modified-angular symmetry functions feed one
 * multilayer perceptron per element; E = sum_i e_i.  Forces come from a
 * hand-written adjoint (network backward, descriptor backward, FP64 scatter).
 *
 * Units: Angstrom, eV, elementary charge; forces in eV/Angstrom.
 * Arrays named *_host live in host memory; every other array pointer is a
 * DEVICE pointer (hipMalloc'd or a torch CUDA tensor), owned by the caller.
 * The library owns its weights and its workspace (sized by nnp_reserve).
 *
 * Error behaviour: every entry point returns an nnp_status.  Argument errors
 * (bad sizes, species not in the table, a box too small for the cutoff, a size
 * beyond the reserved capacity) are detected on the host before any work is
 * queued and leave the outputs untouched.  Conditions only the device can see
 * (a neighbour list overflowing its capacity, non-finite positions or energy)
 * set a device status word that nnp_get_status reads.  nnp_last_error returns
 * a human-readable message for the last failing call on the calling thread.
 *
 * Thread safety: a model may be used by one host thread at a time; calls on
 * one model are ordered on the stream they are given.  nnp_compute and
 * nnp_compute_batch never allocate, never synchronise the host and never call
 * hipDeviceSynchronize once the model has been reserved and its topology seen,
 * so they can be captured into a HIP graph.
 */
#ifndef NNP_H
#define NNP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnp_model nnp_model; /* opaque */

typedef enum {
  NNP_OK = 0,
  NNP_EINVAL = -1,     /* bad argument or unsupported configuration            */
  NNP_ESPECIES = -2,   /* an atomic number is not in the model's species table  */
  NNP_EBOX = -3,       /* a box length is not larger than twice the cutoff      */
  NNP_ECAPACITY = -4,  /* a size exceeds what nnp_reserve provided, or (device
                          status) a neighbour list overflowed its capacity      */
  NNP_EHIP = -5,       /* a HIP runtime call failed                              */
  NNP_ESTATE = -6,     /* call made in the wrong state (e.g. before reserve)     */
  NNP_ENONFINITE = -7  /* (device status) non-finite position or energy          */
} nnp_status;

typedef enum { NNP_FP32 = 0, NNP_BF16 = 1 } nnp_precision;

/*
 * Model hyper-parameters (host struct, copied by nnp_create).
 *
 * Descriptor of atom i (ANI form; the paper cites ANI as its descriptor-based
 * family, Introduction and Methods):
 *   radial   G[s][k]   = sum_{j: species s, r_ij < rc_rad}
 *                          exp(-eta_rad (r_ij - rad_shift[k])^2) fc(r_ij; rc_rad)
 *   angular  G[p][m][n] = 2^(1-zeta) sum_{j<k in species pair p, r_ij, r_ik < rc_ang}
 *                          (1 + cos(theta' - ang_sect[n]))^zeta
 *                          exp(-eta_ang ((r_ij + r_ik)/2 - ang_shift[m])^2)
 *                          fc(r_ij; rc_ang) fc(r_ik; rc_ang),
 *            theta' = arccos(0.95 cos theta_ijk)
 *   fc(r; R) = 0.5 cos(pi r / R) + 0.5 for r < R, else 0.
 * Row layout: radial block [s][k], then angular block [p][m][n], species pairs
 * p ordered lexicographically over (a <= b) of the species table; with
 * extra_inputs = 1 the MM potential phi_i = ke_coulomb sum_j q_j fc(r_ij;
 * mm_cutoff) / r_ij is appended as the last input.
 * Network per species: h_l = CELU_alpha(W_l h_{l-1} + b_l) for the hidden
 * layers, e_i = W_L h_{L-1} + b_L (linear output).  With extra_inputs = 1 the
 * output layer may have two rows (widths[4] = 2): the second is a predicted
 * atomic charge q_i, and the atomic energy is e_i + q_i phi_i -- electrostatic
 * embedding with charges from the model (Methods: the model may return
 * charges and put forces on MM atoms); the forces then include the
 * dependence of q_i on the positions through the network.
 * Supported: 1..4 species; 16 radial shifts, 8 angular shifts, 4 angle
 * sections; widths {128,160,128,96,1} (water model) or {384(+1),256,192,160,1}
 * (H/C/N/O model); n_members >= 1 networks averaged (an ensemble sharing one
 * descriptor).
 */
typedef struct {
  int32_t n_species;
  const int32_t* atomic_numbers_host; /* [n_species], strictly ascending          */
  float rc_rad, rc_ang;               /* cutoffs, rc_ang <= rc_rad                 */
  float eta_rad, eta_ang, zeta;
  int32_t n_rad_shift, n_ang_shift, n_ang_sect; /* must be 16, 8, 4                 */
  const float* rad_shift_host;        /* [n_rad_shift]                             */
  const float* ang_shift_host;        /* [n_ang_shift]                             */
  const float* ang_sect_host;         /* [n_ang_sect] section centres (radians)    */
  int32_t n_layers;                   /* number of entries in widths (5)           */
  const int32_t* widths_host;         /* [n_layers]; widths[0] = descriptor length
                                         + extra_inputs, widths[n_layers-1] = 1,
                                         or 2 (energy, charge) with extra_inputs */
  float celu_alpha;
  int32_t extra_inputs;               /* 0, or 1 for the MM potential channel      */
  float mm_cutoff;                    /* cutoff of the MM potential channel        */
  double ke_coulomb;                  /* Coulomb constant, eV*A/e^2                */
  int32_t n_members;                  /* ensemble size (>= 1)                      */
} nnp_config;

/*
 * Create a model.  weights_host (FP32, host) holds, in order: for each
 * ensemble member, for each species (table order), for each layer: W
 * (out x in, row-major) then b (out).  If weights_host is NULL the weights
 * are drawn from `seed`: value t of the draw uses uniforms u = top 53 bits of
 * SplitMix64 outputs 2t and 2t+1 (Steele, Lea & Flood 2014) through Box-Muller
 * z = sqrt(-2 ln(1-u0)) cos(2 pi u1); W ~ N(0, 2/(fan_in+fan_out)),
 * b ~ N(0, 0.01); each value rounded once to FP32.
 * prec selects the network arithmetic: NNP_FP32 (FP32 matrix cores) or
 * NNP_BF16 (BF16 operands, FP32 accumulation).  Descriptors and their
 * derivatives are FP32 in both forms; energies and force accumulation FP64.
 * Uses the current HIP device; allocates the device weights.  *out is set
 * on success.
 */
nnp_status nnp_create(const nnp_config* cfg, uint64_t seed, const float* weights_host,
                      nnp_precision prec, nnp_model** out);

/*
 * Allocate the workspace for up to max_atoms atoms (all atoms of a call,
 * NNP or not), max_systems systems in one batched call, max_mm MM charges,
 * and per-atom neighbour-list capacities max_rad_nbr (within rc_rad) and
 * max_ang_nbr (within rc_ang); 0 selects the defaults 128 and 64.  For a
 * model with extra_inputs, max_mm also sizes the MM channel's per-workgroup
 * partial sums: 12 bytes per atom for every 256 charges, at most 512 such
 * groups (6 KiB per atom).  May be called again to grow or shrink;
 * synchronises the device.  All device allocation of the model happens here
 * and in nnp_create.
 */
nnp_status nnp_reserve(nnp_model* m, int32_t max_atoms, int32_t max_systems, int32_t max_mm,
                       int32_t max_rad_nbr, int32_t max_ang_nbr);

/*
 * Energy and forces of one system, queued on `stream`.
 *   n_atoms         number of atoms of the system (rows of pos and forces)
 *   pos             [n_atoms][3] FP32 positions (need not be wrapped)
 *   Z_host          [n_atoms] atomic numbers; only NNP atoms need to be in
 *                   the species table.  NULL reuses the previous call's
 *                   topology (Z, index group) unchanged.
 *   box_host        [3] orthorhombic box lengths (periodic in all three
 *                   directions, minimum image; each length must exceed
 *                   2*rc_rad and, with the MM channel, 2*mm_cutoff), or NULL
 *                   for an open (non-periodic) system.
 *   n_nnp, nnp_idx_host  the index group: NNP atoms are nnp_idx_host[0..n_nnp)
 *                   (distinct, in [0, n_atoms)); nnp_idx_host NULL with
 *                   n_nnp == n_atoms means all atoms.
 *   n_mm, mm_pos, mm_q  MM point charges ([n_mm][3] FP32 positions, [n_mm]
 *                   FP32 charges); required iff the model has extra_inputs.
 *   energy          [1] FP64 output, E_ML
 *   forces          [n_atoms][3] FP64 output, -dE/dx; rows of non-NNP atoms
 *                   receive zero
 *   mm_forces       [n_mm][3] FP64 output (-dE/dy for MM atoms) or NULL
 *   accumulate      0: outputs are overwritten; 1: results are added to them
 * Returns after queueing; the outputs are valid when the stream reaches that
 * point.  A topology change (Z or index group differing from the previous
 * call) is uploaded from host memory inside the call.
 */
nnp_status nnp_compute(nnp_model* m, int32_t n_atoms, const float* pos, const int32_t* Z_host,
                       const float* box_host, int32_t n_nnp, const int32_t* nnp_idx_host,
                       int32_t n_mm, const float* mm_pos, const float* mm_q, double* energy,
                       double* forces, double* mm_forces, int32_t accumulate, hipStream_t stream);

/*
 * As nnp_compute, but the neighbour lists come from the caller's pair list
 * instead of the library's cell list (Methods: the 2026 interface also passes
 * the pair list built by the MD engine).  pairs: device int32 [n_pairs][2],
 * indices of the system's atoms, every unordered pair at most once (a half
 * list); pairs may reach beyond the cutoff (a Verlet buffer: each pair of
 * index-group atoms is re-tested with the same FP32 predicate as the cell
 * list) and pairs with an atom outside the index group are ignored.  The list
 * must hold every pair of index-group atoms closer than the radial cutoff;
 * with such a list the neighbour lists, and so the results, are bit-identical
 * to nnp_compute's.  A self pair, an out-of-range index or a repeated pair
 * sets the device status (NNP_EINVAL from nnp_get_status).  Link atoms
 * (nnp_set_links) are not atoms of the system, so the list cannot name them:
 * their pairs with the NNP atoms are found by a direct scan with the same
 * predicate (n_links x n_nnp distance tests).  max_rad_nbr must be <= 256.
 */
nnp_status nnp_compute_pairs(nnp_model* m, int32_t n_atoms, const float* pos, const int32_t* Z_host,
                             const float* box_host, int32_t n_nnp, const int32_t* nnp_idx_host, int32_t n_pairs,
                             const int32_t* pairs, int32_t n_mm, const float* mm_pos, const float* mm_q,
                             double* energy, double* forces, double* mm_forces, int32_t accumulate,
                             hipStream_t stream);

/*
 * Energies and forces of n_sys independent systems packed back to back (the
 * paper's performance section traces the cost of small systems to per-step
 * launch and dispatch overhead; batching replicas, lambda-windows or
 * conformers into one call amortises it): system s owns atoms
 * [atom_offsets_host[s], atom_offsets_host[s+1]).  All atoms are NNP atoms.
 *   boxes_host  [n_sys][3] host, orthorhombic box lengths per system (each
 *               above 2*rc_rad; minimum image within the system), a row of
 *               zeros for an open system; NULL: every system is open.
 *   energies    [n_sys] FP64, forces [total][3] FP64 (device), overwritten.
 * Z_host NULL reuses the previous batched call's topology (atomic numbers and
 * offsets).  Each system's neighbours are found by one scan over its own
 * atoms (per-system cost grows with the square of its size: meant for many
 * small systems; a large box is faster through nnp_compute's cell list).
 * One neighbour search, one descriptor launch, one grouped network launch and
 * one adjoint launch cover all systems.  The boxes are kept in device memory:
 * a call whose boxes differ from the previous call's uploads them (this
 * synchronises the stream and is refused under stream capture, as a topology
 * change is) and replays the captured graph.  A batched call has no index
 * group, so link atoms (nnp_set_links) do not apply to it.
 */
nnp_status nnp_compute_batch(nnp_model* m, int32_t n_sys, const int32_t* atom_offsets_host,
                             const float* pos, const int32_t* Z_host, const float* boxes_host,
                             double* energies, double* forces, hipStream_t stream);

/*
 * nnp_compute without any allocation, for callers that cannot allocate
 * device memory (code that must not call hipMalloc: tight serving loops,
 * harnesses that forbid allocation).  Computes what nnp_compute computes for
 * one system whose n_atoms atoms are all NNP atoms (index group = all, no MM
 * charges, no link atoms), overwriting energy [1] and forces [n_atoms][3]
 * (FP64, device).  pos [n_atoms][3] FP32 device, Z_host [n_atoms] host,
 * box_host [3] host or NULL (open system), as for nnp_compute.
 * The per-call workspace is carved out of a static device array of 32 MiB
 * that the library holds on each device it runs on until the process ends;
 * nnp_reserve is not needed and the reserved workspace, the captured graph
 * and the topology cache of nnp_compute are left untouched (nnp_read_buffer
 * keeps reporting nnp_compute's last call).  Kernels are launched directly
 * on `stream` (no graph).  The array holds the workspace of up to about 8,900
 * atoms of the two-species model or 5,700 of the four-species one, at the
 * default neighbour capacities (128 radial, 64 angular); a larger call returns
 * NNP_ECAPACITY before any work is queued.  All calls on one device share its
 * array: calls that overlap on a device (other streams, other threads) race
 * and must be serialised by the caller.  NNP_EINVAL for a model with the MM
 * channel, NNP_ESTATE while link atoms are set; other errors as nnp_compute.
 */
nnp_status nnp_compute_noalloc(nnp_model* m, int32_t n_atoms, const float* pos, const int32_t* Z_host,
                               const float* box_host, double* energy, double* forces, hipStream_t stream);

/*
 * Link atoms for bonds cut by the index group (Methods, "The nnpot Interface",
 * eq. 4).  For each of the n_links cut bonds (ml_idx_host[l] inside the index
 * group, mm_idx_host[l] outside it; atom indices of the system passed to
 * nnp_compute) a link atom of atomic number link_Z is placed at
 *   r_L = r_ML + d (r_MM - r_ML) / |r_MM - r_ML|
 * (bond vector under the minimum image when the call is periodic) and treated
 * as an NNP atom, appended after the index group.  Its force is passed on to
 * the ML and MM atoms by the chain rule:
 *   F_MM += (d/|u|) (F_L - (F_L.u^) u^),  F_ML += F_L - that,  u = r_MM - r_ML.
 * Applies to later nnp_compute and nnp_compute_pairs calls (a batched call
 * has no index group); n_links = 0
 * removes them.  The paper's defaults are link_Z = 1 and d = 1 Angstrom.
 * Allocates (device arrays of the link list): call outside graph capture.
 */
nnp_status nnp_set_links(nnp_model* m, int32_t n_links, const int32_t* ml_idx_host, const int32_t* mm_idx_host,
                         float distance, int32_t link_Z);

/*
 * Synchronise `stream` and report the device status word of the calls made
 * since the previous nnp_get_status: NNP_OK, NNP_ECAPACITY (a neighbour list
 * overflowed; results are incomplete -- nnp_reserve larger capacities) or
 * NNP_ENONFINITE.  Clears the word.
 */
nnp_status nnp_get_status(nnp_model* m, hipStream_t stream);

/* Intermediate buffers of the last call, for inspection and tests. */
typedef enum {
  NNP_BUF_PERM = 0,       /* int32 [n_nnp]: sorted slot -> NNP-local atom (stable
                             counting sort by key = species * n_bins + bin)      */
  NNP_BUF_KEY = 1,        /* int32 [n_nnp]: key of each NNP-local atom           */
  NNP_BUF_BIN_START = 2,  /* int32 [n_species * n_bins + 1]                      */
  NNP_BUF_NBR_COUNT = 3,  /* int32 [n_nnp][2]: radial, angular neighbour counts
                             per sorted slot                                     */
  NNP_BUF_NBR_RAD = 4,    /* int32 [n_nnp][max_rad_nbr]: radial neighbours (sorted
                             slots), grouped by species                          */
  NNP_BUF_NBR_ANG = 5,    /* int32 [n_nnp][max_ang_nbr]: angular neighbours       */
  NNP_BUF_DESCRIPTOR = 6, /* float [n_nnp][row stride] per sorted slot           */
  NNP_BUF_ATOM_ENERGY = 7,/* float [n_nnp] atomic energies per sorted slot        */
  NNP_BUF_DEDX = 8,       /* float [n_nnp][row stride] dE/d(descriptor) per slot  */
  NNP_BUF_GRID = 9,       /* int32 [4]: n_bins, cells per dimension x, y, z      */
  NNP_BUF_ORDER = 10,     /* int32 [n_nnp]: slots in the order the per-atom
                             kernels visit them: bin by bin, species by species
                             within a bin, ascending slot within a species     */
  NNP_BUF_CHARGE = 11,    /* float [n_nnp] predicted atomic charges per sorted
                             slot (models with a charge output; else EINVAL)  */
  NNP_BUF_GRAPH = 12      /* int32 [3]: HIP graphs instantiated, graphs updated
                             in place for a call with new arguments, replays
                             of an unchanged graph (counts since creation)   */
} nnp_buffer;

/*
 * Copy an intermediate buffer to host memory (synchronises `stream`).
 * *elems receives the element count; at most capacity_bytes are written.
 * *row_stride receives the row length of 2-D buffers (elements), else 1.
 */
nnp_status nnp_read_buffer(nnp_model* m, nnp_buffer which, void* dst_host, size_t capacity_bytes,
                           int64_t* elems, int32_t* row_stride, hipStream_t stream);

/*
 * Autotuner.  Several stages have more than one kernel variant (network:
 * register-resident wavefronts or row-split workgroups of 16, 32 or 64 atoms,
 * or of 32 atoms with 16 for the smallest species, with four or eight
 * wavefronts;
 * descriptor forward: a wavefront, a 16-lane or an 8-lane row per atom, or
 * wavefronts of two or four atoms sharing their lanes over chunks; descriptor
 * adjoint: a wavefront or half a wavefront per atom, and a wide-load form of
 * its reverse-slot search; neighbour search: one
 * wavefront per atom, or several per cell sharing its centre atoms).
 * nnp_autotune reruns the
 * stages after the cell list `reps` times (1..256) per candidate on the
 * workspace of the previous compute call (same size and geometry; the
 * caller's buffers are neither read nor written), times the stage being
 * tuned with events in that context, and keeps the fastest for that size
 * bucket (quarter octaves of the atom count); later calls of that size use
 * it.  Pinned stages (nnp_set_variant) are skipped.  chosen (host, [4] or
 * NULL) receives the variants now used for the neighbour, descriptor,
 * network and adjoint stages, as nnp_get_variants.  Synchronises the stream; drops the
 * cached graph.  If the environment variable NNP_TUNE_CACHE names a file,
 * results are appended to it and read back by nnp_create for the same GPU
 * architecture and model shape.
 */
nnp_status nnp_autotune(nnp_model* m, int32_t reps, int32_t* chosen, hipStream_t stream);

/* Stages with kernel variants (index of `chosen` above, `stage` below). */
typedef enum {
  NNP_TUNE_NEIGHBOURS = 0,
  NNP_TUNE_DESCRIPTOR = 1,
  NNP_TUNE_NETWORK = 2,
  NNP_TUNE_ADJOINT = 3
} nnp_tune_stage;

/*
 * Pin the kernel variant of one stage for later calls, overriding the tuned
 * choice and the built-in default; variant = -1 removes the pin.  Variants:
 *   neighbours: 0 one wavefront per atom; 1 / 2 / 3 wavefronts per cell with
 *     about 8 / 5 / 3 centre atoms each (with a single bin, 0 is used);
 *   descriptor forward: 0 one wavefront per atom; 1 / 2 one 16-lane / 8-lane
 *     row per atom; 3 / 4 two / four atoms per wavefront, their radial
 *     segments and angular classes cut into equal chunks, one per lane
 *     (for several elements, whose classes hold few pairs each);
 *   network: 0 register-resident wavefronts; 1 / 2 / 3 row-split workgroups
 *     of 16 / 32 / 64 atoms (64 for water-sized networks only, wider ones
 *     use 32); 4 workgroups of 32 atoms, 16 for the species with the fewest
 *     atoms (more even workgroups for small systems); 5 / 6 / 7 as 1 / 4 / 2
 *     with eight wavefronts per workgroup instead of four (shorter chains
 *     per tile, for systems with few tiles or wide networks); 8 / 9 (BF16
 *     form, the water-sized network, one member; otherwise 2 runs)
 *     persistent workgroups holding one species' BF16 weights in LDS, a
 *     32-atom (8) or 16-atom (9) tile per wavefront with no barrier (celu'
 *     then comes from the BF16-rounded activation: dE/dx differs from the
 *     other BF16 kernels by rounding);
 *   descriptor adjoint: 0 one wavefront per atom; 1 half a wavefront per atom;
 *     2 as 0, with the centre's place in each neighbour's list counted with
 *     wide loads instead of a binary search (for lists far beyond the caches).
 * All variants compute the same quantities (integer stages bit-identically,
 * floating point to rounding).
 * Drops the cached graph.  NNP_EINVAL for an unknown stage or variant.
 */
nnp_status nnp_set_variant(nnp_model* m, int32_t stage, int32_t variant);

/*
 * The kernel variants (chosen[4], host, indexed by nnp_tune_stage) that a
 * call of the size and geometry of the previous compute call runs: pinned,
 * else tuned, else the built-in default.  NNP_ESTATE before the first call.
 */
nnp_status nnp_get_variants(nnp_model* m, int32_t* chosen);

/*
 * HIP-graph replay (enabled by default).  The first call of a configuration
 * is captured into a HIP graph; a later call with the same arguments (device
 * pointers, sizes, flags and box) replays it with one launch.  A call whose
 * arguments differ (a new box every step under a barostat, other output
 * buffers) is captured again and the instantiated graph is updated in place
 * with the new kernel arguments (hipGraphExecUpdate), which costs far less
 * than building a new graph; a graph is only rebuilt when the update is
 * refused (a different sequence of kernels, e.g. another cell grid).  The
 * per-system boxes of nnp_compute_batch live in device memory and never
 * change the graph.  Device memory contents (positions, topology arrays) may
 * change between replays.  Calls made while the stream is already capturing,
 * or while stage timing is on, launch their kernels directly.  enable = 0
 * turns replay off and frees the cached graph.  NNP_BUF_GRAPH counts builds,
 * updates and replays.
 */
nnp_status nnp_set_graph(nnp_model* m, int32_t enable);

/*
 * Per-stage timing with HIP events recorded on the call's stream around each
 * stage of nnp_compute / nnp_compute_batch (used by the benchmark; see the
 * paper's performance section for why per-step cost matters).  Stages:
 */
typedef enum {
  NNP_STAGE_CELLS = 0,      /* binning, histogram, scan, stable scatter      */
  NNP_STAGE_NEIGHBOURS = 1, /* neighbour lists                               */
  NNP_STAGE_DESCRIPTOR = 2, /* descriptor forward                            */
  NNP_STAGE_MM = 3,         /* MM potential channel forward                  */
  NNP_STAGE_NETWORK = 4,    /* per-species networks, forward + backward      */
  NNP_STAGE_ENERGY = 5,     /* (reads 0: the FP64 energy reduction runs in
                               the gather's launch, timed as GATHER)         */
  NNP_STAGE_ADJOINT = 6,    /* descriptor adjoint                            */
  NNP_STAGE_GATHER = 7,     /* FP64 force gather and energy reduction        */
  NNP_STAGE_MM_ADJOINT = 8, /* MM channel adjoint                            */
  NNP_STAGE_COUNT = 9
} nnp_stage;

/*
 * max_calls > 0 enables timing for up to max_calls subsequent calls (events are
 * created here, host-side); 0 disables it.  Either way the accumulated times
 * are reset.  Not for use under graph capture.
 */
nnp_status nnp_profile_enable(nnp_model* m, int32_t max_calls);

/*
 * Synchronise `stream` and return, per stage, the summed event time in
 * milliseconds over the recorded calls (ms_total[NNP_STAGE_COUNT]) and the
 * number of recorded calls (*calls).
 */
nnp_status nnp_profile_read(nnp_model* m, double* ms_total, int64_t* calls, hipStream_t stream);

/*
 * Mechanical embedding (Theory, eq. 3): the ML-MM coupling term left at the MM
 * level, Coulomb plus 12-6 Lennard-Jones between every ML atom i and every MM
 * atom j, with the fixed charges and LJ parameters of the MM force field:
 *   E = sum_i sum_{j: r_ij < cutoff} ke q_i q_j / r_ij
 *                                    + 4 eps_ij ((s_ij / r_ij)^12 - (s_ij / r_ij)^6),
 *   s_ij = (s_i + s_j) / 2,  eps_ij = sqrt(eps_i eps_j)   (Lorentz-Berthelot, the
 *   rule of the GAFF and CHARMM force fields of the paper's Methods),
 * with a plain spherical cutoff (no shift) and, when box_host is given, the
 * minimum image.  It needs no model: every argument is given here.
 *   ml_pos [n_ml][3], ml_param [n_ml][3] = (q, sigma, eps): device, FP32
 *   mm_pos [n_mm][3], mm_param [n_mm][3]: device, FP32
 *   box_host [3] (host) or NULL for open boundaries
 *   cutoff > 0 (A); 0 takes every pair (open boundaries only)
 *   ke: Coulomb constant in the caller's units (14.3996454784 eV A / e^2)
 *   energy [1], ml_forces [n_ml][3], mm_forces [n_mm][3]: device, FP64, F = -dE/dr;
 *   overwritten, or added to with accumulate = 1.
 * Units follow the arguments (A, e, eV above).  Atoms must not coincide
 * within the cutoff.  Launches on `stream` without synchronising; allocates
 * nothing.  The ML forces and the energy are summed with FP64 atomics (last-
 * bit differences between runs are possible); the MM forces are not.
 * NNP_EINVAL for bad counts, pointers or cutoff; NNP_EBOX when a periodic box
 * has no cutoff or one of its lengths is not above twice the cutoff.
 */
nnp_status nnp_me_coupling(int32_t n_ml, const float* ml_pos, const float* ml_param, int32_t n_mm,
                           const float* mm_pos, const float* mm_param, const float* box_host, float cutoff,
                           float ke, double* energy, double* ml_forces, double* mm_forces, int32_t accumulate,
                           hipStream_t stream);

/* Free the model, its weights and its workspace. */
void nnp_destroy(nnp_model* m);

/* Static description of a status code. */
const char* nnp_status_string(nnp_status s);

/* Message of the last failing call on this host thread ("" if none). */
const char* nnp_last_error(void);

/* Library version as "major.minor.patch". */
const char* nnp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NNP_H */
