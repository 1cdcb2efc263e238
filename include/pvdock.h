/*
 * pvdock.h -- C ABI of the MI355X (gfx950) docking hot path of PocketVina
 * (arXiv 2506.20043): grid maps over the pocket boxes of one receptor, score
 * and analytic gradient of ligand poses, and Monte Carlo + RILC-BFGS search.
 *
 * Conventions shared by every call
 *   - Status: 0 = PV_OK; negative = error.  Nothing throws or aborts across
 *     the ABI.  pv_last_error() returns a thread-local message for the last
 *     failure on the calling thread.
 *   - Host validation happens before anything is enqueued: an invalid call
 *     returns an error and enqueues nothing.
 *   - "host" pointers are read during the call only; "device" pointers must
 *     stay valid until the work enqueued on `stream` has completed.
 *   - Every call is asynchronous and ordered on `stream` (a hipStream_t;
 *     NULL = the null stream).  Results are valid after synchronisation.
 *   - Opaque handles are owned by the library until their *_free call.
 *   - Output buffers are caller-allocated device memory.
 *   - Arithmetic is IEEE binary32.
 *
 * Atom types are the Vina XS types: 0 C_H, 1 C_P, 2 N_P, 3 N_D, 4 N_A,
 * 5 O_A, 6 O_DA, 7 S_P.
 */
#ifndef PVDOCK_H
#define PVDOCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PV_OK = 0,
    PV_E_INVALID = -1,     /* malformed argument (NULL, bad type, bad bond, ...) */
    PV_E_RANGE = -2,       /* size beyond a documented limit */
    PV_E_NOMEM = -3,       /* device or host allocation failed */
    PV_E_DEVICE = -4,      /* a HIP call failed */
    PV_E_UNSUPPORTED = -5, /* request the library does not implement */
    PV_E_STATE = -6        /* handles from different contexts, freed handle, ... */
} pv_status;

#define PV_NTYPES 8
#define PV_MAX_ATOMS 128   /* heavy atoms per ligand */
#define PV_MAX_TORS 32     /* rotatable bonds per ligand */
#define PV_MAX_PAIRS 8128  /* intra pairs per ligand (128 choose 2) */

/* message of the last failure on this thread ("" if none) */
const char* pv_last_error(void);
/* ABI version: major * 100 + minor */
int32_t pv_version(void);

/* ------------------------------------------------------------------ context */
typedef struct pv_ctx pv_ctx;
/* Binds a context to HIP device `device`.  Every later call on the context
 * makes that device current. */
pv_status pv_create(int32_t device, pv_ctx** out);
void pv_destroy(pv_ctx* ctx);

/* ---------------------------------------------------------------- grid maps
 * Grid cache of the paper's "Kernel 1" (Methods, Accelerated Docking;
 * Supplementary Algorithm 2, first step): for every search box and every
 * ligand atom type t, the lattice map
 *     M_t(g) = sum over receptor atoms r with |g - x_r| < 8 A of phi_{t,type_r}(|g - x_r|)
 * where phi is the Vina-form pair energy (gauss1, gauss2, repulsion,
 * hydrophobic, hydrogen bond of the surface distance).  The 8 A test is
 * r < 8 on binary64 values (g = origin + h (i, j, k) and r from the binary32
 * receptor coordinates, each operation rounded to binary64); the terms
 * themselves are binary32.
 *
 * Lattice of a box: n = ceil(size/spacing) + 1 points per axis, origin =
 * binary32(center - (n-1) * spacing / 2) rounded once from binary64, points
 * origin + spacing * (i, j, k).  Maps are [box][type][z][y][x] binary32,
 * resident in device memory and owned by the handle.
 *
 * rec_xyz: host [n_rec][3]; rec_type: host [n_rec], values < 8.
 * boxes: host [n_boxes]; size > 0, spacing > 0, at most 2048 points per axis
 * and fewer than 2^24 points per box (a cube of 255 points: edges up to 95 A at
 * 0.375 A), else PV_E_RANGE.
 * penalty_slope: kcal/mol per A added for each atom coordinate outside a box
 * (its lookups clamp to the box face); must be >= 0.
 * n_rec may be 0 (all maps zero).  Every lattice point sums its receptor
 * atoms in input order, so a build and every rebuild give the same maps bit
 * for bit. */
typedef struct {
    float center[3];
    float size[3];
    float spacing;
} pv_box;

/* Host only (no device needed): the lattice of one box as pv_build_grids
 * defines it. */
pv_status pv_box_lattice(const pv_box* box, int32_t dims[3], float origin[3]);

typedef struct pv_grids pv_grids;
pv_status pv_build_grids(pv_ctx* ctx, int32_t n_rec, const float* rec_xyz, const uint8_t* rec_type,
                         const pv_box* boxes, int32_t n_boxes, float penalty_slope,
                         void* stream, pv_grids** out);
/* dims, origin and the device address of the 8 maps of one box */
pv_status pv_grids_info(const pv_grids* g, int32_t box, int32_t dims[3], float origin[3],
                        const float** dev_maps);
/* recomputes every map from the receptor the handle was built with (the
 * same kernel as pv_build_grids, no allocation), ordered on `stream` */
pv_status pv_grids_rebuild(pv_grids* g, void* stream);
/* copies the 8 maps of one box ([8][nz][ny][nx] binary32) into the caller's
 * device buffer `dst`, ordered on `stream` */
pv_status pv_grids_copy(const pv_grids* g, int32_t box, float* dst, void* stream);
void pv_grids_free(pv_grids* g);

/* ------------------------------------------------------------------ ligands
 * Ligand model of the POT conformation (Eq. qvina_eq_1): rigid fragments
 * are the components left after cutting the rotatable bonds and form a tree;
 * torsion k is the k-th rotatable bond in input order; the root fragment is
 * the largest (ties: the one holding the lowest atom index); the translation
 * is the world position of the root fragment's centroid; psi = 0 is the input
 * geometry and positive psi turns the child (away-from-root) side right-
 * handedly about the axis parent atom -> child atom.  Intra pairs (the
 * e_intra of Eq. qvina_eq_3) are atoms in different fragments at least four
 * bonds apart.
 *
 * Arrays are host, concatenated over ligands: atom_off [n_lig+1], ref_xyz
 * [atoms][3], type [atoms]; bond_off [n_lig+1], bonds [bonds][2] with
 * ligand-local atom indices, rotatable [bonds] (0/1).  Each ligand must be
 * connected, every rotatable bond must be a bridge, and n_atoms <= 128,
 * rotatable bonds <= 32.  Rings are allowed inside fragments.  PV_E_RANGE if
 * a concatenated device table (pairs, force-slot table) would pass 2^31
 * entries. */
typedef struct pv_ligands pv_ligands;
pv_status pv_ligands_create(pv_ctx* ctx, int32_t n_lig, const int32_t* atom_off, const float* ref_xyz,
                            const uint8_t* type, const int32_t* bond_off, const int32_t* bonds,
                            const uint8_t* rotatable, pv_ligands** out);
/* info = {n_atoms, n_frag, n_tors, n_pairs, root_size, depth, dof (7+T), 0} */
pv_status pv_ligands_info(const pv_ligands* l, int32_t lig, int32_t info[8]);
void pv_ligands_free(pv_ligands* l);

/* Host only (no device needed): checks one ligand and describes the model
 * pv_ligands_create would build.  info as pv_ligands_info.  pairs (may be
 * NULL): the intra pairs as [n_pairs][2] input atom indices, lower index
 * first, at most max_pairs of them (PV_E_RANGE if more).  frag (may be NULL):
 * [n_atoms] fragment of each input atom, 0 = root, in the depth-first order
 * of the torsion tree. */
pv_status pv_ligand_describe(int32_t n_atoms, const float* ref_xyz, const uint8_t* type, int32_t n_bonds,
                             const int32_t* bonds, const uint8_t* rotatable, int32_t info[8], int32_t* pairs,
                             int32_t max_pairs, int32_t* frag);

/* --------------------------------------------------------------- score+grad
 * Score SF = e_inter + e_intra (Eq. qvina_eq_3) of B poses and its analytic
 * gradient.  e_inter is the trilinear interpolation of the box's map of each
 * atom's type plus the out-of-box penalty; e_intra sums the pair energy over
 * the ligand's intra pairs closer than 8 A.
 *
 * dof: device [B][dof_stride], row = [tx, ty, tz, qw, qx, qy, qz, psi_0 ..
 * psi_{T-1}] (the quaternion need not be unit; a zero quaternion gives NaN).
 * lig_of_pose, box_of_pose: device [B]; an out-of-range index sets that
 * pose's outputs to NaN.
 * grad_energy: device [B] upstream factor for a backward pass, or NULL (= 1).
 * Outputs (device, any may be NULL):
 *   energy [B]; e_parts [B][2] = (e_inter, e_intra);
 *   grad_dof [B][dof_stride]: grad_energy * dSF/d(t, q, psi), where the
 *   quaternion part is the derivative with respect to the raw input q;
 *   xyz_out, grad_xyz [B][xyz_stride][3]: atom coordinates and
 *   grad_energy * dSF/dx in the caller's atom order; rows past the pose's
 *   ligand's atoms are 0, and every row of an out-of-range pose is NaN.
 * dof_stride >= 7 + max T; xyz_stride >= max atoms when xyz outputs are used. */
pv_status pv_score_grad(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, int32_t n_poses,
                        const int32_t* lig_of_pose, const int32_t* box_of_pose, const float* dof,
                        int32_t dof_stride, const float* grad_energy, float* energy, float* e_parts,
                        float* grad_dof, float* xyz_out, float* grad_xyz, int32_t xyz_stride,
                        void* stream);

/* The same score on given world coordinates xyz [B][xyz_stride][3] (caller's
 * atom order): energy, e_parts and grad_energy * dSF/dx. */
pv_status pv_score_grad_xyz(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, int32_t n_poses,
                            const int32_t* lig_of_pose, const int32_t* box_of_pose, const float* xyz,
                            int32_t xyz_stride, const float* grad_energy, float* energy, float* e_parts,
                            float* grad_xyz, void* stream);

/* -------------------------------------------------------------------- search
 * Parameters of RILC-BFGS (Eqs. qvina_eq_6 .. qvina_eq_12) and of the Monte
 * Carlo chains (Supplementary Algorithm 2).  BFGS runs in the 6+T tangent
 * space (translation, rotation vector, torsions) with the orientation moved
 * by a left rotation; Lewis-Overton line search with Armijo parameter ls_rho
 * and weak-Wolfe parameter ls_sigma, at most ls_max_trials trials starting
 * from step 1; cautious update when y.s/s.s > eps_curv * |g|; history of
 * bfgs_m pairs; stop when |g| <= eps_grad, when the direction is not a
 * descent direction, or after bfgs_max_iter iterations.
 * MC step: mutate one entity (position by a uniform point of a ball of
 * radius mut_pos_amp; orientation by a uniform rotation vector of a ball of
 * radius mut_rot_amp / R_g; or one torsion redrawn), BFGS, Metropolis
 * acceptance exp((e_cur - e_new) / temperature), and a new best refined by a
 * second BFGS of at most refine_max_iter iterations.
 * consistency = 1 gates the step's BFGS with the first-order consistency
 * check (Eqs. qvina_eq_4 and qvina_eq_5): the mutated pose is compared with
 * the current pose, its neighbour, in the tangent coordinates the mutation
 * moved (translation, rotation vector, or the one torsion).  BFGS runs when
 * in one of them the derivative changes sign between the two poses or
 * disagrees with the secant slope; otherwise the step ends after that one
 * evaluation, with no optimisation and no Metropolis move.
 * Random numbers: Philox4x64-10 keyed (seed, 0) with counter (block, step,
 * chain, job). */
typedef struct {
    int32_t chains;          /* MC chains per job, >= 1 */
    int32_t steps;           /* MC steps per chain, >= 0 */
    int32_t bfgs_max_iter;   /* >= 0 */
    int32_t bfgs_m;          /* 1 .. 8 */
    int32_t ls_max_trials;   /* 1 .. 64 */
    int32_t refine_max_iter; /* >= 0 */
    float ls_rho, ls_sigma, eps_grad, eps_curv;
    float temperature, mut_pos_amp, mut_rot_amp;
    uint32_t flags;          /* PV_DOCK_* */
    uint64_t seed;
    int32_t workgroups;      /* persistent launch width; 0 = chosen by the library */
    int32_t consistency;     /* 0: every step runs BFGS (default); 1: the consistency check gates it */
    int64_t max_evals;       /* evaluation budget per chain, >= 0; 0 = none.  A chain whose count
                                reaches it after a step stops there (status PV_JOB_BUDGET) */
} pv_dock_params;

/* Per-chain and per-job status bits of a dock (0 = ok).  Failures never stop
 * the other chains or jobs. */
#define PV_JOB_NONFINITE 1u   /* job: the best energy is not finite */
#define PV_JOB_BUDGET 2u      /* chain: stopped at max_evals; job: some chain did */
#define PV_JOB_OUTSIDE 4u     /* chain: its best pose has an atom outside the box (its energy carries
                                 the out-of-box penalty); job: the best chain's pose does */

#define PV_DOCK_TIMESTAMPS 1u /* write per-job device timestamps */
#define PV_DOCK_GRAPH 2u      /* pv_dock_run captures its launches in a hipGraph once and replays it */
/* hand out each size class's jobs most costly ligand first (an evaluation's
 * energy work: 8 x pairs + 48 x atoms + 109 x torsions; ties keep the job
 * order), so that short chains fill the end of the launch.  Only the order in
 * which chains start changes: every chain's result depends on (seed, job,
 * chain) alone, so the outputs are identical bit for bit. */
#define PV_DOCK_LARGEST_FIRST 4u
/* hand out each size class's jobs grouped by box (ascending box index; inside
 * a box, the job order, or the PV_DOCK_LARGEST_FIRST order when that flag is
 * set too), so that the chains in flight at any time read one or two boxes'
 * maps and the L2 caches hold those instead of every box's.  As with
 * PV_DOCK_LARGEST_FIRST only the start order changes: outputs are identical
 * bit for bit. */
#define PV_DOCK_BOX_ORDER 8u
/* every line-search trial runs its pair loop: the intra lower-bound check
 * (see chain_bounded) is off.  The check only ever rejects trials the full
 * energy rejects, so the searches, energies, poses and evaluation counts are
 * identical bit for bit; chain_bounded is zero and chain_pairs counts every
 * trial's pairs.  For checking that claim and timing the check. */
#define PV_DOCK_NO_INTRA_BOUND 16u
/* other flag bits are rejected (PV_E_INVALID) */

/* fills the defaults: 30 BFGS iterations, m = 5, 10 trials, rho 1e-4,
 * sigma 0.1, eps_grad 1e-3, eps_curv 1e-6, temperature 1.2, amplitudes 2 A */
void pv_dock_params_default(pv_dock_params* p);

typedef struct { int32_t ligand, box; } pv_job;

/* Outputs of a dock (device arrays; any may be NULL):
 *   chain_best_e [jobs*chains], chain_best_dof [jobs*chains][dof_stride],
 *   chain_evals [jobs*chains] (score+grad evaluations, line-search trials
 *   and refinements included), chain_pairs [jobs*chains] (intra pairs
 *   evaluated inside the cutoff, summed over the evaluations that ran the
 *   pair loop),
 *   job_best_e [jobs], job_best_chain [jobs] (ties: lowest chain),
 *   job_evals [jobs], job_status [jobs] (PV_JOB_* bits, 0 = ok),
 *   job_t_start, job_t_end [jobs] (device clock, 100 MHz; with
 *   PV_DOCK_TIMESTAMPS), chain_grads [jobs*chains] (the evaluations that
 *   computed the gradient: a line-search trial above the sufficient-decrease
 *   bound stops after its energy, since no step reads its gradient),
 *   chain_status [jobs*chains] (PV_JOB_BUDGET, PV_JOB_OUTSIDE bits),
 *   chain_bounded [jobs*chains] (line-search trials decided before the pair
 *   loop: their map energy plus a lower bound of the intra energy -- each
 *   pair's class's least pair energy, summed -- is already above the
 *   sufficient-decrease bound, so the full energy is too; they are counted
 *   in chain_evals, not in chain_grads, and add no pairs; the gather
 *   variants only: the slot variant always runs the pair loop and leaves
 *   zeros).  The outside test
 *   re-evaluates each chain's best pose once at its end; that evaluation is
 *   not counted in chain_evals. */
typedef struct {
    float* chain_best_e;
    float* chain_best_dof;
    int64_t* chain_evals;
    int64_t* chain_pairs;
    float* job_best_e;
    int32_t* job_best_chain;
    int64_t* job_evals;
    int32_t* job_status;
    uint64_t* job_t_start;
    uint64_t* job_t_end;
    int32_t dof_stride;
    int64_t* chain_grads;
    int32_t* chain_status;
    int64_t* chain_bounded;
} pv_dock_out;

/* A dock plan: the job table uploaded once and the parameters checked.
 * jobs: host [n_jobs]; every ligand and box index must exist.  A chain's
 * result depends only on the inputs, the parameters and (job, chain): runs
 * of a plan, graph replays, the plain form, the schedule's width and the job
 * order all give the same outputs bit for bit (the kernel variant may sum
 * forces in another order). */
typedef struct pv_plan pv_plan;
pv_status pv_dock_plan(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, const pv_job* jobs,
                       int32_t n_jobs, const pv_dock_params* params, pv_plan** out);
/* Batched form: every (job, chain) of the plan in one persistent launch
 * whose waves pull work from a device queue (plus a reset and a per-job
 * reduction).  Captured in a hipGraph when the plan's flags ask for it. */
pv_status pv_dock_run(pv_plan* plan, const pv_dock_out* out, void* stream);
/* Plain form: one launch per job, in job order, on `stream`
 * (the per-ligand loop of Supplementary Algorithm 2). */
pv_status pv_dock_run_plain(pv_plan* plan, const pv_dock_out* out, void* stream);
void pv_plan_free(pv_plan* plan);

/* Schedules.  A plan splits its jobs into size classes (ligands of at most
 * 64 atoms first, larger ones second; classes without jobs are left out),
 * and each class runs one persistent launch of pv_dock_run.  Its schedule:
 * the kernel variant (PV_VARIANT_*, below), the launch width in one-wave
 * workgroups and, reported only, the dynamic LDS bytes per workgroup, the
 * workgroups one CU holds and the class's job count.  The plan starts from
 * the occupancy model of pv_launch_info; pv_dock_run_plain always uses that
 * model for its per-job launches. */
typedef struct {
    int32_t variant;
    int32_t workgroups;
    int32_t lds_bytes;
    int32_t per_cu;
    int32_t n_jobs;
} pv_schedule;
pv_status pv_plan_groups(const pv_plan* plan, int32_t* n_groups);
pv_status pv_plan_schedule(const pv_plan* plan, int32_t group, pv_schedule* out);
/* Sets a class's variant and width.  PV_VARIANT_SLOTS and PV_VARIANT_GATHER
 * need ligands of at most 64 atoms; PV_VARIANT_GATHER2 takes any.  A
 * workgroup of the variant must fit a CU (PV_E_RANGE otherwise); workgroups
 * 0 = all the CUs hold at once, else 1 .. jobs x chains of the class.  Drops
 * a captured graph (the next pv_dock_run captures again). */
pv_status pv_plan_set_schedule(pv_plan* plan, int32_t group, int32_t variant, int32_t workgroups);

/* Autotuner of the batched launch.  For every size class it times each
 * candidate schedule -- every variant legal for the class, at widths of 1,
 * 3/4 and 1/2 of the workgroups the CUs hold (capped by the class's work) --
 * on a short run of the class's launch (tune_steps >= 1 Monte Carlo steps per
 * chain, outputs to the plan's own scratch, no timestamps) over the class's
 * first jobs in the order the launch hands them out (enough chains to fill
 * the widest candidate 8 times, or the whole class when it has fewer), keeps
 * the best of `repeats` >= 1 timings (HIP events on `stream`) and sets the candidate
 * with the most evaluations per second; on a tie the earlier candidate (the
 * model's schedule comes first) wins.  The choice is remembered by the
 * context, keyed by the class's ligand limits, work items, tune_steps and
 * search settings, and a later call on a plan of the same key takes it
 * without timing (reported with cached = 1); it keeps the latest 256 such
 * choices.  results: host, up to
 * max_results entries (may be NULL); n_results: how many were written (may
 * be NULL).  Synchronises `stream`; drops a captured graph.  Calls that
 * overlap on one plan race; the context's memory of choices is locked. */
typedef struct {
    int32_t group, variant, workgroups;
    int32_t chosen;    /* 1 for the candidate the class now runs */
    int32_t cached;    /* 1 when taken from the context without timing */
    float ms;          /* best timing of the short run (0 when cached) */
    double evals_per_s;
} pv_tune_result;
pv_status pv_dock_autotune(pv_plan* plan, int32_t tune_steps, int32_t repeats, void* stream,
                           pv_tune_result* results, int32_t max_results, int32_t* n_results);

/* plan + batched run + free in one call; it synchronises `stream` before
 * it releases the plan, so it returns after the dock has completed */
pv_status pv_dock(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, const pv_job* jobs,
                  int32_t n_jobs, const pv_dock_params* params, const pv_dock_out* out, void* stream);

/* Allocation-free dock, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, checks and outputs as pv_dock (host jobs,
 * device outputs), and the same outputs bit for bit: the jobs are split
 * into the same size classes, each run by one persistent launch with the
 * variant and width pv_dock_plan would choose.  It calls no hipMalloc,
 * hipFree or other allocating routine: the job table, the per-class job
 * maps, the queue counters and, when chain_best_e or chain_evals is NULL,
 * those per-chain arrays live in one file-scope device array per GPU
 * (about 12.8 MB, held from the first pv_create on that GPU until the
 * process ends).  Limits: n_jobs <= PV_NOALLOC_MAX_JOBS and n_jobs x chains
 * <= PV_NOALLOC_MAX_CHAINS (PV_E_RANGE otherwise).  Only the
 * PV_DOCK_TIMESTAMPS flag is accepted (PV_E_INVALID for others).  Every call
 * on a GPU shares that GPU's array, which keeps the last call's contents:
 * calls on one device are serialised by a lock in the library and each
 * returns only after its work has completed on `stream`, so calls from
 * several host threads of one process do not overlap; anything else that
 * wrote the array while a call ran would race with it. */
#define PV_NOALLOC_MAX_JOBS 65536
#define PV_NOALLOC_MAX_CHAINS 1048576
pv_status pv_dock_noalloc(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, const pv_job* jobs,
                          int32_t n_jobs, const pv_dock_params* params, const pv_dock_out* out, void* stream);

/* Local optimisation only: one BFGS run (the parameters' bfgs_* and ls_*
 * fields) from each of B poses.  dof_in, dof_out: device [B][dof_stride];
 * energy [B]; n_evals [B] (may be NULL).  dof_out quaternions are unit. */
pv_status pv_local_opt(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, int32_t n_poses,
                       const int32_t* lig_of_pose, const int32_t* box_of_pose, const float* dof_in,
                       int32_t dof_stride, const pv_dock_params* params, float* dof_out, float* energy,
                       int64_t* n_evals, void* stream);

/* Output stage (Methods, end of "Accelerated Docking with QuickVina 2-GPU
 * 2.1"; the last steps of Supplementary Algorithm 2): per job, the chains'
 * best poses are taken in ascending energy (ties to the lower chain, NaN
 * last) and clustered greedily: a pose is kept unless its heavy-atom
 * r.m.s.d. (same atom order) to a kept pose is below rmsd_cut, up to
 * `modes` poses.  Each kept pose is refined by BFGS (refine_max_iter
 * iterations with the plan's BFGS settings; the receptor is rigid) and
 * rescored: its energy E = e_inter + e_intra and the reported affinity
 * e_inter / (1 + affinity_w T).  The refined poses are sorted by E (ties to
 * the earlier kept pose), filtered by r.m.s.d. the same way, and written in
 * that order.  One wave per job.
 *
 * plan: the jobs, grids, ligands, chains and BFGS settings of a dock plan.
 * chain_best_e [n_jobs][chains], chain_best_dof [n_jobs][chains][in_stride]:
 * device, typically a pv_dock_out of that plan after pv_dock_run.
 * Outputs (device, caller-owned): n_modes [n_jobs]; per job `modes`
 * entries of mode_chain (source chain, -1 past n_modes), mode_e,
 * mode_affinity (may be NULL) (NaN past n_modes) and mode_dof (may be NULL;
 * [n_jobs][modes][dof_stride], unit quaternion, zero past n_modes and past
 * 7 + T).  Limits: modes 1..PV_MAX_MODES, chains <= PV_MAX_OUTPUT_CHAINS,
 * and the LDS of one workgroup (PV_E_RANGE). */
#define PV_MAX_MODES 32
#define PV_MAX_OUTPUT_CHAINS 4096
typedef struct {
    int32_t modes;           /* poses returned per job at most (the paper samples 20) */
    int32_t refine_max_iter; /* BFGS iterations refining each kept pose; 0 = none */
    float rmsd_cut;          /* A; returned poses are at least this far apart */
    float affinity_w;        /* affinity = e_inter / (1 + affinity_w * torsions) */
} pv_output_params;
void pv_output_params_default(pv_output_params* p);   /* 20, 30, 1.0, 0.0585 */
typedef struct {
    int32_t* n_modes;
    int32_t* mode_chain;
    float* mode_e;
    float* mode_affinity;
    float* mode_dof;
    int32_t dof_stride;
} pv_modes_out;
pv_status pv_output_stage(pv_plan* plan, const float* chain_best_e, const float* chain_best_dof,
                          int32_t in_stride, const pv_output_params* params, const pv_modes_out* out,
                          void* stream);

/* ------------------------------------------------------- receptor surface
 * The step before the path (Methods, "Pocket prediction with P2Rank"):
 * points on the receptor's solvent-accessible surface and the per-point
 * features of Eq. prank_eq_1.
 *
 * pv_sas_build: for every atom a and unit direction u_k (host dirs
 * [n_dirs][3]) the candidate c = x_a + r_a u_k, r_a = X-Score radius of a's
 * XS type + probe, each coordinate one binary32 fused multiply-add; a
 * candidate is dropped when it lies strictly inside another atom's
 * expanded sphere (binary32 fma(dx,dx,fma(dy,dy,dz*dz)) < r_b*r_b).  The
 * kept points are numbered in (atom, direction) order.  Host inputs; the
 * call synchronises `stream` once (it reads the point count back).
 * pv_sas_copy: device xyz [n][3] and atom [n] (either may be NULL); with
 * no points, pv_sas_copy and pv_sas_features write nothing and accept NULL.
 * pv_sas_features: device features [n][12]: channels 0..7 the one-hot XS
 * type, 8..10 the hydrophobic, donor and acceptor flags, each summing
 * max(0, 1 - d/6) over atoms with d^2 < 36; channel 11 the protrusion, the
 * number of atoms with d^2 < 100 (binary32 decisions as above). */
#define PV_MAX_SAS_DIRS 4096
typedef struct pv_sas pv_sas;
pv_status pv_sas_build(pv_ctx* ctx, int32_t n_rec, const float* rec_xyz, const uint8_t* rec_type, int32_t n_dirs,
                       const float* dirs, float probe, void* stream, pv_sas** out);
pv_status pv_sas_info(const pv_sas* sas, int32_t* n_points);
pv_status pv_sas_copy(const pv_sas* sas, float* xyz, int32_t* atom, void* stream);
pv_status pv_sas_features(const pv_sas* sas, float* features, void* stream);
void pv_sas_free(pv_sas* sas);

/* Launch shape diagnostics (host only, no device work): the kernel variant
 * that a launch of `kind` over `items` waves (dock: jobs x chains; score and
 * local-opt: poses) on these ligands uses, its dynamic LDS bytes per
 * workgroup and how many of its workgroups one CU holds.  Variants:
 *   PV_VARIANT_SLOTS    one atom per lane; each intra pair writes its force
 *                       into slots of its two atoms' rows in LDS;
 *   PV_VARIANT_GATHER   one atom per lane; per-pair coefficients in LDS, an
 *                       atom -> pair table in global memory;
 *   PV_VARIANT_GATHER2  two atoms per lane (ligands over 64 atoms), gather.
 * Slots are chosen while they still let the CUs hold as many of the
 * launch's waves as the gather layout would.  Any output may be NULL. */
#define PV_KIND_DOCK 0
#define PV_KIND_SCORE 1
#define PV_KIND_LOCAL_OPT 2
#define PV_VARIANT_SLOTS 0
#define PV_VARIANT_GATHER 1
#define PV_VARIANT_GATHER2 2
pv_status pv_launch_info(pv_ctx* ctx, const pv_ligands* ligs, int32_t kind, int64_t items, int32_t* variant,
                         int32_t* lds_bytes, int32_t* per_cu);

/* Measurement aid (not part of docking): the FP32 VALU issue rate of the
 * device, for comparing the published vector peak with what hand-written
 * FP32 code built here can reach.  Launches n_out threads (a positive
 * multiple of 256) that each run 16 independent multiply-add chains for
 * `iters` rounds, with no memory traffic but one store of their sum to
 * dev_out [n_out] (device, caller-owned).  One launch performs
 * 2 * 16 * iters * n_out floating-point operations; time it on `stream`.
 * PV_E_INVALID for NULL dev_out, iters < 1 or a bad n_out. */
pv_status pv_fma_peak(pv_ctx* ctx, int32_t iters, float* dev_out, int32_t n_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif
