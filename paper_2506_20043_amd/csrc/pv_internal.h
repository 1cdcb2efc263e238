// pv_internal.h -- device-side data layouts shared by the host library and
// the gfx950 kernels of the docking hot path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace pv {

constexpr int kNTypes = 8;
constexpr int kMaxAtoms = 128;
constexpr int kMaxTors = 32;
constexpr int kMaxFrag = kMaxTors + 1;
constexpr int kWave = 64;

// Per-ligand header in device memory.  Atoms are stored in depth-first
// fragment order (each torsion moves one contiguous atom range); fragments
// in depth-first preorder with the root first.
struct alignas(16) DevLig {
    int32_t atom_base, n_atoms, frag_base, n_frag;
    int32_t pair_base, n_pairs, tors_base, n_tors;
    int32_t rounds;      // pointer-doubling rounds to compose the frame tree
    int32_t ell_base;    // first word of the atom -> pair table
    int32_t ell_w;       // entries per atom row (the largest row)
    int32_t pad0;
    float anchor[3];     // reference centroid of the root fragment
    float rot_amp_scale; // 1 / max(R_g, 1e-3)
};

// One rigid fragment.  Fragment 0 is the root (parent -1).
struct alignas(16) DevFrag {
    int32_t parent;      // parent fragment (local index), -1 at the root
    int32_t tors;        // torsion joining it to its parent (input order), -1 at the root
    int32_t child_atom;  // child-side atom of that torsion (local, new order)
    int32_t a0;          // first atom of the fragment (local, new order)
    int32_t sub_end;     // one past the last atom of its subtree
    int32_t pad0, pad1, pad2;
    float axis[4];       // unit axis parent atom -> child atom, reference frame
    float xc[4];         // reference position of the child-side atom
};

// Intra pair packed as i | j << 8 | rk << 16 | class << 24 (new atom order; the
// radius-sum code fills byte 2 alone, so the kernel converts it in one step).
// Atom record: x, y, z and w = bits(type | fragment << 8).
// pslot (same index as the pair list): the slot the pair occupies in the
// row of its first atom | in the row of its second atom << 16 (force-slot
// layout: slot s of atom a at s * (n | 1) + a, slots below ell_w).
// Atom -> pair table (ELL, [n][ell_w] words, rows 16-byte aligned): entry k of atom i is
// p | j << 16, the k-th pair p (index into the pair list) that holds atom i
// and its partner j; rows shorter than ell_w are padded with p = n_pairs
// (a zero coefficient) and j = i.

// Host model of one ligand (built by build_ligand_model).
struct LigModel {
    int n = 0, nf = 0, nt = 0, np = 0, depth = 0, rounds = 0, root_size = 0;
    std::vector<int> perm;          // new -> input atom index
    std::vector<float> ref;         // [n][4] new order: x, y, z, w-bits
    std::vector<DevFrag> frags;     // preorder
    std::vector<int> tors_frag;     // torsion k -> fragment
    std::vector<uint32_t> pairs;    // i | j << 8 | rk << 16 | class << 24 (radius sum 3.4 + 0.1 rk;
                                    // class 0 plain, 1 hydrophobic, 2 hydrogen bond), grouped by class
    std::vector<uint32_t> ell;      // [n][ell_w]
    std::vector<uint32_t> pslot;    // per pair: slot in row i | slot in row j << 16
    int ell_w = 0;
    float anchor[3] = {0, 0, 0};
    float rg = 0.f;
};

// Returns 0 or a negative pv_status; `err` names the problem.
int build_ligand_model(int n, const float* xyz, const uint8_t* type, int nb, const int32_t* bonds,
                       const uint8_t* rot, LigModel& out, std::string& err);


// ------------------------------------------------------------ launchers
struct GridDev {
    const float* maps;    // [box][8][nz][ny][nx]
    const int32_t* dims;  // [box][4] nx, ny, nz, pad
    const float* geom;    // [box][8] ox, oy, oz, h, inv_h, ext_x, ext_y, ext_z
    const int64_t* map_off; // [box] offset of the box's first map
    int32_t n_boxes;
    float kappa;
};

struct LigDev {
    const DevLig* ligs;
    const float4* atoms;
    const int16_t* perm;
    const DevFrag* frags;
    const int8_t* tors_frag;
    const uint32_t* pairs;
    const uint32_t* ell;
    const uint32_t* pslot;   // indexed like pairs
    int32_t n_lig;
    int32_t max_atoms, max_pairs, max_tors;
    int32_t max_ell;   // largest ell_w * n_atoms
};

struct ScoreArgs {
    GridDev g;
    LigDev l;
    int32_t n_poses;
    const int32_t* lig_of_pose;
    const int32_t* box_of_pose;
    const float* dof;      // or xyz when from_xyz
    int32_t dof_stride;
    int32_t from_xyz;
    const float* grad_energy;
    float* energy;
    float* e_parts;
    float* grad_dof;
    float* xyz_out;
    float* grad_xyz;
    int32_t xyz_stride;
};

// the PV_DOCK_NO_INTRA_BOUND bit of the ABI's dock flags (SearchParams::flags)
constexpr uint32_t kDockNoIntraBound = 16u;

struct SearchParams {
    int32_t chains, steps, max_iter, m, ls_max, refine_max_iter;
    float rho, sigma, eps_g, eps_c, temperature, pos_amp, rot_amp;
    uint32_t flags;
    int32_t consistency;   // 1: the first-order consistency check gates the step's BFGS
    uint64_t seed;
    int64_t max_evals;     // evaluation budget per chain (0: none)
};

struct DockArgs {
    GridDev g;
    LigDev l;
    SearchParams sp;
    const int2* jobs;         // (ligand, box)
    int32_t n_jobs;
    int32_t job_begin;        // first job of this launch
    int64_t n_items;          // (job, chain) items of this launch
    uint32_t* queue;          // work counter (persistent launch)
    const int32_t* job_map;   // persistent launch: item / chains -> job (NULL: job_begin + item / chains)
    int32_t persistent;
    // outputs
    float* chain_best_e;
    float* chain_best_dof;
    int64_t* chain_evals;
    int64_t* chain_pairs;
    int64_t* chain_grads;     // evaluations that computed the gradient
    int64_t* chain_bounded;   // trials decided by their map energy and the intra lower bound
    int32_t* chain_status;    // PV_JOB_BUDGET / PV_JOB_OUTSIDE bits per chain (never NULL)
    uint64_t* job_t_start;
    uint64_t* job_t_end;
    int32_t dof_stride;
};

struct OptArgs {
    GridDev g;
    LigDev l;
    SearchParams sp;
    int32_t n_poses;
    const int32_t* lig_of_pose;
    const int32_t* box_of_pose;
    const float* dof_in;
    int32_t dof_stride;
    float* dof_out;
    float* energy;
    int64_t* n_evals;
};

struct OutputArgs {
    GridDev g;
    LigDev l;
    SearchParams sp;          // BFGS settings of the refinement
    const int2* jobs;         // (ligand, box)
    int32_t n_jobs, chains;
    const float* chain_e;     // [n_jobs][chains]
    const float* chain_dof;   // [n_jobs][chains][in_stride]
    int32_t in_stride;
    int32_t modes, refine_max_iter;
    float rmsd_cut, affinity_w;
    int32_t* n_modes;         // [n_jobs]
    int32_t* mode_chain;      // [n_jobs][modes]
    float* mode_e;
    float* mode_affinity;
    float* mode_dof;          // [n_jobs][modes][out_stride]
    int32_t out_stride;
};

struct GridBuildArgs {
    const float4* atoms;      // per box: receptor atoms near the box (x, y, z, w = type bits)
    const int32_t* atom_off;  // [box+1]
    float* maps;
    const int64_t* map_off;
    const int32_t* dims;
    const float* geom;
    const int32_t* tile_off;  // [box+1] first tile of each box
    int32_t n_boxes;
};

hipError_t launch_build_grids(const GridBuildArgs& a, int64_t n_tiles, hipStream_t s);
// Kernel variant of a launch: 0 = one atom per lane with LDS force slots,
// 1 = one atom per lane with the coefficient gather, 2 = two atoms per lane
// with the coefficient gather; lds = dynamic LDS bytes per workgroup and
// per_cu = workgroups one CU holds at once.
struct LaunchShape {
    int variant;
    int lds;
    int per_cu;
};
enum KernelKind { kKindDock = 0, kKindScore = 1, kKindOpt = 2 };
hipError_t launch_shape(int kind, const LigDev& l, int64_t items, int n_cu, LaunchShape* out);
// The shape of one given variant (0 and 1 need ligands of at most 64 atoms);
// hipErrorInvalidConfiguration when no workgroup of it fits a CU.
hipError_t launch_shape_variant(int kind, const LigDev& l, int variant, LaunchShape* out);

hipError_t launch_score(const ScoreArgs& a, int n_cu, hipStream_t s);
hipError_t launch_dock(const DockArgs& a, const LaunchShape& sh, int32_t workgroups, hipStream_t s);
hipError_t launch_reset_queue(uint32_t* q, hipStream_t s);
hipError_t launch_fma_peak(float* out, int n, int iters, hipStream_t s);
hipError_t launch_job_reduce(const float* chain_best_e, const int64_t* chain_evals, const int32_t* chain_status,
                             int32_t n_jobs, int32_t chains, float* job_best_e, int32_t* job_best_chain,
                             int64_t* job_evals, int32_t* job_status, hipStream_t s);
hipError_t launch_local_opt(const OptArgs& a, int n_cu, hipStream_t s);
hipError_t launch_output(const OutputArgs& a, hipStream_t s);
hipError_t launch_sas_candidates(const float4* atoms, int n_rec, const float* dirs, int n_dirs, float probe,
                                 int64_t n_cand, float4* cand, uint8_t* keep, int32_t* block_count, hipStream_t s);
hipError_t launch_sas_scatter(const float4* cand, const uint8_t* keep, const int32_t* block_offset, int64_t n_cand,
                              float4* pts, hipStream_t s);
hipError_t launch_sas_features(const float4* atoms, int n_rec, const float4* pts, int n_pts, float* feat,
                               hipStream_t s);
int sas_block_size();
int output_lds_bytes(const LigDev& l, int chains, int modes);
hipError_t launch_reset_times(uint64_t* t0, uint64_t* t1, int n, hipStream_t s);

// Scratch of the allocation-free dock entry point, one file-scope device
// array per GPU (see noalloc_scratch): the queue counters of the two size
// classes, the job table, the per-class job maps and, for callers that take
// no per-chain outputs, the chains' best energies, evaluation counts and
// statuses.
constexpr int64_t kNoAllocMaxJobs = 65536;
constexpr int64_t kNoAllocMaxChains = 1 << 20;   // jobs x chains
struct NoAllocLayout {
    uint32_t* queues;   // [2]
    int2* jobs;         // [kNoAllocMaxJobs]
    int32_t* map;       // [kNoAllocMaxJobs]: class 0 jobs, then class 1 jobs
    float* best;        // [kNoAllocMaxChains]
    int64_t* evals;     // [kNoAllocMaxChains]
    int32_t* status;    // [kNoAllocMaxChains]
};
constexpr size_t kNoAllocOffJobs = 256;
constexpr size_t kNoAllocOffMap = kNoAllocOffJobs + 8 * kNoAllocMaxJobs;
constexpr size_t kNoAllocOffBest = kNoAllocOffMap + 4 * kNoAllocMaxJobs;
constexpr size_t kNoAllocOffEvals = kNoAllocOffBest + 4 * kNoAllocMaxChains;
constexpr size_t kNoAllocOffStatus = kNoAllocOffEvals + 8 * kNoAllocMaxChains;
constexpr size_t kNoAllocBytes = kNoAllocOffStatus + 4 * kNoAllocMaxChains;
inline NoAllocLayout noalloc_layout(void* base)
{
    char* b = (char*)base;
    return {(uint32_t*)b, (int2*)(b + kNoAllocOffJobs), (int32_t*)(b + kNoAllocOffMap),
            (float*)(b + kNoAllocOffBest), (int64_t*)(b + kNoAllocOffEvals), (int32_t*)(b + kNoAllocOffStatus)};
}
// Device address of the current device's scratch array, looked up once per
// device (hipGetSymbolAddress with that device current) and kept.
hipError_t noalloc_scratch(void** out);
// Fills the per-class job maps in job order (ligands of at most 64 atoms
// first, from map[0]; larger ones from map[n_small]) and zeroes both queue
// counters.  One workgroup.
hipError_t launch_class_map(const int2* jobs, int32_t n_jobs, const DevLig* ligs, int32_t n_small, int32_t* map,
                            uint32_t* queues, hipStream_t s);

// Tiles of the grid-map kernel.
constexpr int kTileX = 16, kTileY = 4, kTileZ = 4;

}  // namespace pv
