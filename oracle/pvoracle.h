/*
 * pvoracle.h -- plain double-precision CPU oracle of the PocketVina docking
 * hot path (arXiv 2506.20043: Methods, "Accelerated Docking with QuickVina
 * 2-GPU 2.1", Eqs. qvina_eq_1 .. qvina_eq_13, and Supplementary Algorithm 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the checker the GPU path is held to.
 * It is not part of the product: only the test suite, the smoke entry and
 * the CPU-baseline leg of the benchmark load it.  It shares no code, header
 * or table with the HIP library.
 *
 * All arithmetic is IEEE binary64.  Receptor coordinates and the lattice
 * origin and spacing are binary32, the precision they have at the interface.
 * The one decision taken in binary32 is the receptor surface point set
 * (or_sas_points), which is compared as a set of integers.
 *
 * Return codes: 0 = OK; negative = invalid input (nothing written).
 */
#ifndef PVORACLE_H
#define PVORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_NTYPES 8

/* ---- scoring terms (Eq. qvina_eq_3; Vina functional form, see oracle.c) */
void   or_terms(double d, double v[5], double dv[5]);
double or_pair(int ta, int tb, double r, double* dphi_dr);
void   or_type_params(int t, double* radius, int* hydrophobic, int* donor, int* acceptor);
void   or_weights(double w[5]);

/* ---- lattice of one search box */
int or_lattice(const double center[3], const double size[3], double h,
               int dims[3], float origin[3]);

/* ---- grid maps: maps[t][k][j][i], t < 8 (Kernel 1); cutoff r < 8 in
 * binary64; margin (may be NULL): per point the smallest |r - 8| */
int or_build_maps(int n_rec, const float* rec_xyz, const int32_t* rec_type,
                  const int dims[3], const float origin[3], float h,
                  double* maps, double* margin);
int or_map_point(int n_rec, const float* rec_xyz, const int32_t* rec_type,
                 const int dims[3], const float origin[3], float h,
                 int i, int j, int k, double out[8], double* margin);

/* ---- trilinear lookup with out-of-box penalty */
double or_trilinear(const double* map, const int dims[3], const float origin[3],
                    float h, double kappa, const double x[3], double grad[3],
                    double* face_dist);

/* ---- ligand model: rigid fragments, torsion tree, intra pair list */
typedef struct or_ligand or_ligand;
int  or_ligand_build(int n_atoms, const double* ref_xyz, const int32_t* type,
                     int n_bonds, const int32_t* bonds, const uint8_t* rotatable,
                     or_ligand** out);
void or_ligand_free(or_ligand* L);
/* info[0..7] = n_atoms, n_frag, n_tors, n_pairs, root_frag, depth, 0, 0 */
void or_ligand_info(const or_ligand* L, int32_t info[8]);
void or_ligand_pairs(const or_ligand* L, int32_t* pairs /* [n_pairs][2] */);
void or_ligand_frag(const or_ligand* L, int32_t* frag /* [n_atoms] */);
/* per torsion: bond index, parent-side atom, child-side atom */
void or_ligand_torsions(const or_ligand* L, int32_t* tors /* [T][3] */);
double or_ligand_rg(const or_ligand* L);
void or_ligand_anchor(const or_ligand* L, double anchor[3]);

/* ---- pose evaluation */
typedef struct {
    double min_face;   /* smallest distance (A) of an atom to a lattice plane or box face */
    double min_cut;    /* smallest |r - 8| over intra pairs */
    double min_kink;   /* smallest |d - kink| over intra pairs with an active hyd / hbond kink */
    int64_t pairs_in;  /* intra pairs inside the cutoff */
} or_flags;

/* grid of one box: 8 maps in double, lattice and penalty slope */
typedef struct {
    const double* maps;   /* [8][nz][ny][nx] */
    int dims[3];
    float origin[3];
    float h;
    double kappa;
} or_grid;

void or_fk(const or_ligand* L, const double* dof, double* xyz);
/* e3 = {E, e_inter, e_intra}; grad_dof [7+T]; grad_tan [6+T] = (dE/dt, torque, dE/dpsi) */
int or_score_grad(const or_ligand* L, const or_grid* G, const double* dof,
                  double e3[3], double* grad_dof, double* grad_tan,
                  double* xyz, double* grad_xyz, or_flags* flags);
int or_score_xyz(const or_ligand* L, const or_grid* G, const double* xyz,
                 double e3[3], double* grad_xyz, or_flags* flags);
double or_inter_pairwise(int n_rec, const float* rec_xyz, const int32_t* rec_type,
                         int n, const double* xyz, const int32_t* type);

/* ---- counter-based RNG: Philox4x64-10 (Salmon et al., SC'11) */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* ---- RILC-BFGS (Eqs. qvina_eq_6 .. qvina_eq_12) */
typedef struct {
    int32_t max_iter, m, ls_max, pad;
    double rho, sigma, eps_g, eps_c;
} or_bfgs_params;
int or_bfgs(const or_ligand* L, const or_grid* G, const or_bfgs_params* P,
            const double* x0, double* xout, double* fout,
            int64_t* n_evals, int32_t* n_iters);

/* x (+) lam d: t + lam d_t, exp(lam d_theta) q (left rotation, renormalised),
 * psi + lam d_psi; x [7+nt], d [6+nt], o [7+nt] */
void or_retract(int nt, const double* x, const double* d, double lam, double* o);

/* The same run, reporting how close its decisions came to going the other
 * way (test infrastructure: a binary32 run may take the other branch of a
 * decision within its rounding).  Dimensionless margins, the smallest over
 * the run:
 *   armijo    |f_t - (f + rho lam g.d)| / (1 + |f_t|) over every trial;
 *   wolfe     |g_t.d - sigma g.d| / (|d|_1 (1 + |g_t|_inf)) over trials that
 *             passed Armijo;
 *   curvature |y.s/s.s - eps_c |g|| / (|y.s/s.s| + eps_c |g|);
 *   descent   |g.d| / (|d|_1 (1 + |g|));
 *   pose      the smallest min(min_face, min_cut, min_kink) of any pose
 *             evaluated (A). */
typedef struct { double armijo, wolfe, curvature, descent, pose; } or_bfgs_margins;
int or_bfgs_margins_run(const or_ligand* L, const or_grid* G, const or_bfgs_params* P,
                        const double* x0, double* xout, double* fout, int64_t* n_evals,
                        int32_t* n_iters, or_bfgs_margins* margins);

/* the same BFGS on a flat R^n objective with an additive update */
typedef void (*or_eval_fn)(void* user, const double* x, double* f, double* g);
int or_bfgs_generic(int n, or_eval_fn fn, void* user, const or_bfgs_params* P,
                    const double* x0, double* xout, double* fout, int64_t* n_evals,
                    int32_t* n_iters);

/* ---- first-order consistency check (Eqs. qvina_eq_4 and qvina_eq_5):
 * 1 (local optimisation warranted) when, for some tangent coordinate p in
 * [p_lo, p_hi), with x the mutated pose (energy fx, tangent gradient gx
 * [6+T]) and y its neighbour (fy, gy),
 *   sign(gx_p) sign(gy_p) <= 0                          (Eq. qvina_eq_4)
 * or, failing that,
 *   sign(gx_p) sign((fx - fy) (x - y)_p) <= 0          (Eq. qvina_eq_5)
 * with (x - y) the tangent difference: translation, the rotation vector of
 * q_x conj(q_y), torsions wrapped to (-pi, pi]. */
int or_consistency_passes(int nt, const double* x, double fx, const double* gx,
                          const double* y, double fy, const double* gy, int p_lo, int p_hi);

/* ---- Monte Carlo chains (Supplementary Algorithm 2) */
typedef struct {
    int32_t chains, steps;
    or_bfgs_params bfgs;
    int32_t refine_max_iter;
    int32_t consistency;   /* 1: the first-order consistency check gates BFGS; 0: every step runs BFGS */
    double temperature, mut_pos_amp, mut_rot_amp;
    uint64_t seed;
} or_mc_params;
int or_init_pose(const or_ligand* L, const or_grid* G, uint64_t seed,
                 int job, int chain, double* dof);
/* one mutation (Eq. qvina_eq_2) of pose x (7 + nt values, in place) from the
 * step's 8 Philox words; for the tests of its distributions */
void or_mutate(const or_ligand* L, const or_mc_params* P, const uint64_t w[8], double* x);
/* the Metropolis decision of a step (Eq. qvina_eq_13): 1 if e_o replaces
 * e_cur, with u = u01(word) */
int or_metropolis_accepts(double e_cur, double e_o, uint64_t word, double temperature);
int or_mc_chain(const or_ligand* L, const or_grid* G, const or_mc_params* P,
                int job, int chain, double* best_dof, double* best_e,
                int64_t* n_evals);
/* jobs [n_jobs][2] = (ligand, grid); chain outputs [n_jobs*chains(*stride)] */
int or_dock(int n_lig, or_ligand* const* ligs, int n_grids, const or_grid* grids,
            int n_jobs, const int32_t* jobs, const or_mc_params* P, int dof_stride,
            int n_threads, double* chain_best_e, double* chain_best_dof,
            int64_t* chain_evals, double* job_best_e, int32_t* job_best_chain);

/* ---- output stage (Methods, end of "Accelerated Docking with QuickVina
 * 2-GPU 2.1"; last steps of Supplementary Algorithm 2): the chains' best
 * poses are clustered and sorted, the selected ones refined and rescored,
 * then r.m.s.d.-filtered and sorted again, and at most `modes` returned.
 * dof [n_chains][7+T], e [n_chains]; outputs [modes] in final order:
 * chain index, energy (e_inter + e_intra of the refined pose), affinity
 * e_inter / (1 + affinity_w T), pose [7+T] with a unit quaternion.
 * margins (may be NULL): [0] smallest |rmsd - rmsd_cut| over the cluster
 * and filter decisions taken, [1] smallest energy gap between neighbours of
 * the final sort. */
typedef struct {
    int32_t modes, refine_max_iter;
    double rmsd_cut, affinity_w;
    or_bfgs_params bfgs;
} or_output_params;
int or_output_stage(const or_ligand* L, const or_grid* G, int n_chains, const double* dof,
                    const double* e, const or_output_params* P, int32_t* n_out,
                    int32_t* out_chain, double* out_e, double* out_aff, double* out_dof,
                    double margins[2]);

/* ---- receptor surface points and point features (the step before the
 * path: Methods, "Pocket prediction with P2Rank", Eq. prank_eq_1).
 * Candidates: for every atom a and direction u_k, c = x_a + r_a u_k with
 * r_a = radius(a) + probe, each coordinate fmaf(r_a, u_k, x_a) in binary32.
 * A candidate is kept unless, for some other atom b,
 * fmaf(dx,dx,fmaf(dy,dy,dz*dz)) < r_b*r_b in binary32 (strictly inside b's
 * expanded sphere).  Kept points in (atom, direction) order.  Returns the
 * number kept (<= cap; -1 on invalid input). */
int or_sas_points(int n_rec, const float* rec_xyz, const int32_t* rec_type, int n_dirs,
                  const float* dirs, float probe, int cap, float* pts, int32_t* atom);
/* Eq. prank_eq_1 per point: channel c of 11 (one-hot XS type 0..7, then
 * hydrophobic, donor, acceptor) sums max(0, 1 - d/6) over atoms with
 * d^2 < 36 (binary32 decision as above); channel 11 (protrusion) counts the
 * atoms with d^2 < 100.  feat [n_pts][12]. */
void or_point_features(int n_rec, const float* rec_xyz, const int32_t* rec_type, int n_pts,
                       const float* pts, double* feat);

#ifdef __cplusplus
}
#endif
#endif
