/*
 * pvoracle.c -- plain double-precision CPU oracle of the PocketVina docking
 * hot path (arXiv 2506.20043).
 *
 * TEST INFRASTRUCTURE ONLY: the checker the HIP path is held to.  Only the
 * test suite, the smoke entry and the CPU-baseline leg of the benchmark may
 * load it; the product never does.  It shares no code with the HIP library.
 *
 * What it follows (section / equation of the paper):
 *   - grid cache, one map per ligand atom type ("Kernel 1", Methods 4.2 and
 *     Supplementary Algorithm 2, first step);
 *   - the POT conformation C = {x,y,z, a,b,c,d, psi_1..psi_Nrot} (Eq. qvina_eq_1);
 *   - the score SF = e_inter + e_intra, e_inter by trilinear interpolation
 *     in the grid cache, e_intra over ligand atom pairs (Eq. qvina_eq_3);
 *   - the jitter mutation R(.) of one POT entity (Eq. qvina_eq_2);
 *   - RILC-BFGS: d = -grad (Eq. qvina_eq_6), Lewis-Overton line search with
 *     the Armijo and weak-Wolfe tests (Eqs. qvina_eq_7, qvina_eq_8), update
 *     (Eqs. qvina_eq_9, qvina_eq_10), cautious curvature test
 *     (Eq. qvina_eq_11), two-loop recursion over the m latest pairs, and
 *     termination on a small gradient or a non-descent direction
 *     (Eq. qvina_eq_12);
 *   - Metropolis acceptance (Eq. qvina_eq_13), best tracking and refinement
 *     of a new best, per-thread best output (Supplementary Algorithm 2).
 *
 * The paper does not define the empirical terms.  They follow the published
 * AutoDock Vina form (Trott & Olson 2010, the scoring function the paper's
 * engine inherits): gauss1, gauss2, repulsion, hydrophobic and hydrogen-bond
 * terms of the surface distance d = r - R_a - R_b, with an 8 A cutoff.
 * Every other reading of a silent or garbled passage is listed where it is
 * used.
 *
 * Plain loops, no blocking or fusion: each function is meant to be checked
 * against its definition by eye.
 */
#include "pvoracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Constants: X-Score radii by element, Vina term weights.             */
/* Types: 0 C_H, 1 C_P, 2 N_P, 3 N_D, 4 N_A, 5 O_A, 6 O_DA, 7 S_P.     */
/* ------------------------------------------------------------------ */
static const double T_RADIUS[OR_NTYPES] = {1.9, 1.9, 1.8, 1.8, 1.8, 1.7, 1.7, 2.0};
static const int    T_HYD[OR_NTYPES]    = {1, 0, 0, 0, 0, 0, 0, 0};
static const int    T_DON[OR_NTYPES]    = {0, 0, 0, 1, 0, 0, 1, 0};
static const int    T_ACC[OR_NTYPES]    = {0, 0, 0, 0, 1, 1, 1, 0};
static const double W_TERM[5] = {-0.0356, -0.00516, 0.840, -0.0351, -0.587};
static const double CUTOFF = 8.0;
static const double PI = 3.14159265358979323846;

void or_type_params(int t, double* radius, int* hyd, int* don, int* acc)
{
    *radius = T_RADIUS[t]; *hyd = T_HYD[t]; *don = T_DON[t]; *acc = T_ACC[t];
}

void or_weights(double w[5]) { for (int i = 0; i < 5; ++i) w[i] = W_TERM[i]; }

/* The five terms of the surface distance d and their derivatives d/dd.
 * gauss1 = exp(-(d/0.5)^2); gauss2 = exp(-((d-3)/2)^2);
 * repulsion = d^2 for d < 0;
 * hydrophobic = 1 below 0.5, linear to 0 at 1.5;
 * hbond = 1 below -0.7, linear to 0 at 0.
 * Interval convention: each linear piece is closed on the left. */
void or_terms(double d, double v[5], double dv[5])
{
    double a = d / 0.5;
    v[0] = exp(-a * a);
    dv[0] = -8.0 * d * v[0];
    double b = (d - 3.0) / 2.0;
    v[1] = exp(-b * b);
    dv[1] = -b * v[1];
    if (d < 0.0) { v[2] = d * d; dv[2] = 2.0 * d; }
    else         { v[2] = 0.0;   dv[2] = 0.0; }
    if (d < 0.5)      { v[3] = 1.0;     dv[3] = 0.0; }
    else if (d < 1.5) { v[3] = 1.5 - d; dv[3] = -1.0; }
    else              { v[3] = 0.0;     dv[3] = 0.0; }
    if (d < -0.7)     { v[4] = 1.0;      dv[4] = 0.0; }
    else if (d < 0.0) { v[4] = -d / 0.7; dv[4] = -1.0 / 0.7; }
    else              { v[4] = 0.0;      dv[4] = 0.0; }
}

static int pair_is_hyd(int a, int b) { return T_HYD[a] && T_HYD[b]; }
static int pair_is_hb(int a, int b)
{
    return (T_DON[a] && T_ACC[b]) || (T_ACC[a] && T_DON[b]);
}

/* phi_ab(r): weighted sum of the terms; the caller applies the cutoff. */
double or_pair(int ta, int tb, double r, double* dphi_dr)
{
    double d = r - T_RADIUS[ta] - T_RADIUS[tb];
    double v[5], dv[5];
    or_terms(d, v, dv);
    int hy = pair_is_hyd(ta, tb), hb = pair_is_hb(ta, tb);
    double e = W_TERM[0] * v[0] + W_TERM[1] * v[1] + W_TERM[2] * v[2];
    double de = W_TERM[0] * dv[0] + W_TERM[1] * dv[1] + W_TERM[2] * dv[2];
    if (hy) { e += W_TERM[3] * v[3]; de += W_TERM[3] * dv[3]; }
    if (hb) { e += W_TERM[4] * v[4]; de += W_TERM[4] * dv[4]; }
    if (dphi_dr) *dphi_dr = de;
    return e;
}

/* ------------------------------------------------------------------ */
/* Lattice: n = ceil(size/h) + 1 points per axis, centred on the box   */
/* centre; the origin is rounded once to binary32, and the lattice is  */
/* g = origin + h * (i, j, k).                                         */
/* ------------------------------------------------------------------ */
int or_lattice(const double center[3], const double size[3], double h,
               int dims[3], float origin[3])
{
    if (!(h > 0.0)) return -1;
    for (int a = 0; a < 3; ++a) {
        if (!(size[a] > 0.0) || !isfinite(center[a]) || !isfinite(size[a])) return -1;
        double n = ceil(size[a] / h) + 1.0;
        if (n > 4096.0) return -2;
        dims[a] = (int)n;
        origin[a] = (float)(center[a] - 0.5 * (double)(dims[a] - 1) * h);
    }
    return 0;
}

static int types_ok(int n, const int32_t* t)
{
    for (int i = 0; i < n; ++i)
        if (t[i] < 0 || t[i] >= OR_NTYPES) return 0;
    return 1;
}

/* Map value of every ligand type at one lattice point: the sum over the
 * receptor atoms closer than the 8 A cutoff, in atom-index order.  The
 * lattice point g = origin + h (i, j, k), the distance and the cutoff test
 * r < 8 are all binary64.  margin (may be NULL): the smallest |r - 8| over
 * all receptor atoms (infinity with none), so that a test can tell the
 * points where a binary32 build may decide the cutoff the other way.
 * (Point-major.) */
int or_map_point(int n_rec, const float* rec, const int32_t* rtype,
                 const int dims[3], const float origin[3], float h,
                 int i, int j, int k, double out[8], double* margin)
{
    if (i < 0 || j < 0 || k < 0 || i >= dims[0] || j >= dims[1] || k >= dims[2]) return -1;
    if (!types_ok(n_rec, rtype)) return -1;
    double g[3] = {(double)origin[0] + (double)h * i, (double)origin[1] + (double)h * j,
                   (double)origin[2] + (double)h * k};
    double mg = INFINITY;
    for (int t = 0; t < OR_NTYPES; ++t) out[t] = 0.0;
    for (int r = 0; r < n_rec; ++r) {
        const float* x = rec + 3 * r;
        double dx = g[0] - x[0], dy = g[1] - x[1], dz = g[2] - x[2];
        double dist = sqrt(dx * dx + dy * dy + dz * dz);
        if (fabs(dist - CUTOFF) < mg) mg = fabs(dist - CUTOFF);
        if (!(dist < CUTOFF)) continue;
        for (int t = 0; t < OR_NTYPES; ++t) out[t] += or_pair(t, rtype[r], dist, NULL);
    }
    if (margin) *margin = mg;
    return 0;
}

/* All maps of one box.  Atom-major: every receptor atom adds its terms to
 * the lattice points inside its cutoff sphere (r < 8 in binary64, as in
 * or_map_point).  Per point, the atoms are still summed in index order, so
 * the result equals or_map_point.  margin (may be NULL): [nz][ny][nx], per
 * point the smallest |r - 8| over the receptor atoms within 8.01 A
 * (infinity with none), as or_map_point's margin wherever it is below
 * 0.01. */
int or_build_maps(int n_rec, const float* rec, const int32_t* rtype,
                  const int dims[3], const float origin[3], float h, double* maps,
                  double* margin)
{
    if (!types_ok(n_rec, rtype)) return -1;
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const size_t plane = (size_t)nx * ny, msz = plane * nz;
    memset(maps, 0, sizeof(double) * msz * OR_NTYPES);
    if (margin)
        for (size_t p = 0; p < msz; ++p) margin[p] = INFINITY;
    const double reach = CUTOFF + 0.01; /* the lattice range scanned per atom */
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < nz; ++k) {
        double gz = (double)origin[2] + (double)h * k;
        for (int r = 0; r < n_rec; ++r) {
            const float* x = rec + 3 * r;
            if (fabs(gz - x[2]) > reach) continue;
            int jlo = (int)ceil((x[1] - reach - origin[1]) / h);
            int jhi = (int)floor((x[1] + reach - origin[1]) / h);
            int ilo = (int)ceil((x[0] - reach - origin[0]) / h);
            int ihi = (int)floor((x[0] + reach - origin[0]) / h);
            if (jlo < 0) jlo = 0;
            if (ilo < 0) ilo = 0;
            if (jhi > ny - 1) jhi = ny - 1;
            if (ihi > nx - 1) ihi = nx - 1;
            for (int j = jlo; j <= jhi; ++j) {
                double gy = (double)origin[1] + (double)h * j;
                for (int i = ilo; i <= ihi; ++i) {
                    double gx = (double)origin[0] + (double)h * i;
                    double dx = gx - x[0], dy = gy - x[1], dz = gz - x[2];
                    double dist = sqrt(dx * dx + dy * dy + dz * dz);
                    size_t idx = (size_t)k * plane + (size_t)j * nx + i;
                    if (margin && fabs(dist - CUTOFF) < margin[idx]) margin[idx] = fabs(dist - CUTOFF);
                    if (!(dist < CUTOFF)) continue;
                    for (int t = 0; t < OR_NTYPES; ++t)
                        maps[t * msz + idx] += or_pair(t, rtype[r], dist, NULL);
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Trilinear interpolation of one map (Eq. qvina_eq_3: e_inter is read  */
/* from the grid cache by trilinear interpolation).                    */
/* f = (x - o)/h per axis, clamped to [0, n-1]; cell i0 = min(floor f,  */
/* n-2); the gradient is the derivative of the interpolant in that cell */
/* (zero along a clamped axis).  Outside the box a penalty kappa times  */
/* the distance to the box is added, with gradient +-kappa.            */
/* ------------------------------------------------------------------ */
double or_trilinear(const double* map, const int dims[3], const float origin[3],
                    float h, double kappa, const double x[3], double grad[3],
                    double* face_dist)
{
    int i0[3];
    double u[3], pen = 0.0, dpen[3] = {0, 0, 0}, fd = INFINITY;
    int clamped[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        double lo = (double)origin[a], hi = lo + (double)h * (dims[a] - 1);
        double f = (x[a] - lo) / (double)h;
        if (x[a] < lo) {
            pen += kappa * (lo - x[a]); dpen[a] = -kappa; f = 0.0; clamped[a] = 1;
            if (lo - x[a] < fd) fd = lo - x[a];
        } else if (x[a] > hi) {
            pen += kappa * (x[a] - hi); dpen[a] = kappa; f = (double)(dims[a] - 1); clamped[a] = 1;
            if (x[a] - hi < fd) fd = x[a] - hi;
        } else {
            double fl = floor(f), dd = (double)h * fmin(f - fl, fl + 1.0 - f);
            if (dd < fd) fd = dd;
        }
        int c = (int)floor(f);
        if (c > dims[a] - 2) c = dims[a] - 2;
        i0[a] = c;
        u[a] = f - c;
    }
    const int nx = dims[0], ny = dims[1];
    double v = 0.0, du[3] = {0, 0, 0};
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                double m = map[((size_t)(i0[2] + cz) * ny + (i0[1] + cy)) * nx + (i0[0] + cx)];
                double wx = cx ? u[0] : 1.0 - u[0];
                double wy = cy ? u[1] : 1.0 - u[1];
                double wz = cz ? u[2] : 1.0 - u[2];
                v += wx * wy * wz * m;
                du[0] += (cx ? 1.0 : -1.0) * wy * wz * m;
                du[1] += wx * (cy ? 1.0 : -1.0) * wz * m;
                du[2] += wx * wy * (cz ? 1.0 : -1.0) * m;
            }
    for (int a = 0; a < 3; ++a)
        grad[a] = (clamped[a] ? 0.0 : du[a] / (double)h) + dpen[a];
    if (face_dist) *face_dist = fd;
    return v + pen;
}

/* ------------------------------------------------------------------ */
/* Ligand model.  Rigid fragments are the connected components left    */
/* after cutting the rotatable bonds; they form a tree whose edges are  */
/* the torsions psi_k of Eq. qvina_eq_1.  Readings:                     */
/*  - torsion k is the k-th rotatable bond in input order;              */
/*  - the root fragment is the largest (ties: lowest fragment id, ids   */
/*    numbered by their lowest atom index);                             */
/*  - psi_k = 0 is the input geometry; positive psi_k turns the child   */
/*    side right-handedly about the axis parent atom -> child atom;     */
/*  - the translation is the world position of the root centroid;       */
/*  - intra pairs ("paired atoms inside the ligand", Eq. qvina_eq_3):   */
/*    i < j in different fragments and at least 4 bonds apart.         */
/* ------------------------------------------------------------------ */
struct or_ligand {
    int n, nb, nf, nt, np, root, depth;
    double* ref;
    int* type;
    int* frag;
    int* tors_bond;
    int* tors_a;        /* parent-side atom */
    int* tors_c;        /* child-side atom */
    int* tors_cfrag;    /* child fragment */
    int* tors_pfrag;    /* parent fragment */
    int* frag_tors;     /* torsion joining a fragment to its parent, -1 at root */
    int* frag_bfs;      /* fragments in breadth-first order from the root */
    unsigned char* sub; /* [nt][n]: atom moves with torsion k */
    int* pairs;         /* [np][2] */
    double anchor[3];
    double rg;
};

void or_ligand_free(or_ligand* L)
{
    if (!L) return;
    free(L->ref); free(L->type); free(L->frag); free(L->tors_bond); free(L->tors_a);
    free(L->tors_c); free(L->tors_cfrag); free(L->tors_pfrag); free(L->frag_tors);
    free(L->frag_bfs); free(L->sub); free(L->pairs);
    free(L);
}

int or_ligand_build(int n, const double* ref, const int32_t* type, int nb,
                    const int32_t* bonds, const uint8_t* rot, or_ligand** out)
{
    *out = NULL;
    if (n < 1 || nb < 0) return -1;
    if (nb < n - 1) return -2; /* cannot be connected; rings are allowed */
    if (!types_ok(n, type)) return -1;
    for (int i = 0; i < 3 * n; ++i)
        if (!isfinite(ref[i])) return -1;
    for (int b = 0; b < nb; ++b) {
        int u = bonds[2 * b], v = bonds[2 * b + 1];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) return -1;
        for (int c = 0; c < b; ++c) {
            int u2 = bonds[2 * c], v2 = bonds[2 * c + 1];
            if ((u == u2 && v == v2) || (u == v2 && v == u2)) return -1;
        }
    }
    /* adjacency (dense: the oracle only meets ligands of <= a few hundred atoms) */
    unsigned char* adj = calloc((size_t)n * n, 1);
    unsigned char* adjr = calloc((size_t)n * n, 1); /* rigid (non-rotatable) bonds */
    int* queue = malloc(sizeof(int) * (n + 1));
    int* dist = malloc(sizeof(int) * n);
    for (int b = 0; b < nb; ++b) {
        int u = bonds[2 * b], v = bonds[2 * b + 1];
        adj[u * n + v] = adj[v * n + u] = 1;
        if (!rot[b]) adjr[u * n + v] = adjr[v * n + u] = 1;
    }
    int rc = 0;
    /* connectivity */
    for (int i = 0; i < n; ++i) dist[i] = -1;
    int qh = 0, qt = 0;
    queue[qt++] = 0; dist[0] = 0;
    while (qh < qt) {
        int u = queue[qh++];
        for (int v = 0; v < n; ++v)
            if (adj[u * n + v] && dist[v] < 0) { dist[v] = dist[u] + 1; queue[qt++] = v; }
    }
    if (qt != n) rc = -2;

    or_ligand* L = calloc(1, sizeof(or_ligand));
    L->n = n; L->nb = nb;
    L->ref = malloc(sizeof(double) * 3 * n);
    L->type = malloc(sizeof(int) * n);
    L->frag = malloc(sizeof(int) * n);
    memcpy(L->ref, ref, sizeof(double) * 3 * n);
    for (int i = 0; i < n; ++i) L->type[i] = type[i];

    /* fragments over rigid bonds, ids in order of their lowest atom */
    int nf = 0;
    for (int i = 0; i < n; ++i) L->frag[i] = -1;
    for (int s = 0; s < n && rc == 0; ++s) {
        if (L->frag[s] >= 0) continue;
        qh = qt = 0; queue[qt++] = s; L->frag[s] = nf;
        while (qh < qt) {
            int u = queue[qh++];
            for (int v = 0; v < n; ++v)
                if (adjr[u * n + v] && L->frag[v] < 0) { L->frag[v] = nf; queue[qt++] = v; }
        }
        ++nf;
    }
    int nt = 0;
    for (int b = 0; b < nb; ++b) nt += rot[b] ? 1 : 0;
    L->nf = nf; L->nt = nt;
    if (rc == 0) {
        for (int b = 0; b < nb; ++b)
            if (rot[b] && L->frag[bonds[2 * b]] == L->frag[bonds[2 * b + 1]]) rc = -3;
        if (nf != nt + 1) rc = -3; /* the fragment graph must be a tree */
    }
    if (rc != 0) { or_ligand_free(L); free(adj); free(adjr); free(queue); free(dist); return rc; }

    /* root: largest fragment, lowest id on ties */
    int* fsize = calloc(nf, sizeof(int));
    for (int i = 0; i < n; ++i) fsize[L->frag[i]]++;
    int root = 0;
    for (int f = 1; f < nf; ++f) if (fsize[f] > fsize[root]) root = f;
    L->root = root;
    free(fsize);

    L->tors_bond = malloc(sizeof(int) * (nt + 1));
    L->tors_a = malloc(sizeof(int) * (nt + 1));
    L->tors_c = malloc(sizeof(int) * (nt + 1));
    L->tors_cfrag = malloc(sizeof(int) * (nt + 1));
    L->tors_pfrag = malloc(sizeof(int) * (nt + 1));
    L->frag_tors = malloc(sizeof(int) * nf);
    L->frag_bfs = malloc(sizeof(int) * nf);
    {
        int k = 0;
        for (int b = 0; b < nb; ++b) if (rot[b]) L->tors_bond[k++] = b;
    }
    /* breadth-first walk of the fragment tree from the root */
    int* fdepth = malloc(sizeof(int) * nf);
    for (int f = 0; f < nf; ++f) { L->frag_tors[f] = -1; fdepth[f] = -1; }
    qh = qt = 0; queue[qt++] = root; fdepth[root] = 0;
    int maxd = 0;
    while (qh < qt) {
        int f = queue[qh++];
        for (int k = 0; k < nt; ++k) {
            int b = L->tors_bond[k];
            int u = bonds[2 * b], v = bonds[2 * b + 1];
            int fu = L->frag[u], fv = L->frag[v], child = -1, pa = -1, ca = -1;
            if (fu == f && fdepth[fv] < 0) { child = fv; pa = u; ca = v; }
            else if (fv == f && fdepth[fu] < 0) { child = fu; pa = v; ca = u; }
            if (child < 0) continue;
            fdepth[child] = fdepth[f] + 1;
            if (fdepth[child] > maxd) maxd = fdepth[child];
            L->frag_tors[child] = k;
            L->tors_a[k] = pa; L->tors_c[k] = ca;
            L->tors_cfrag[k] = child; L->tors_pfrag[k] = f;
            queue[qt++] = child;
        }
    }
    for (int f = 0; f < nf; ++f) L->frag_bfs[f] = queue[f];
    L->depth = maxd;
    free(fdepth);

    /* atoms moved by each torsion: every atom whose fragment lies below it */
    L->sub = calloc((size_t)(nt > 0 ? nt : 1) * n, 1);
    for (int i = 0; i < n; ++i) {
        int f = L->frag[i];
        while (f != root) {
            int k = L->frag_tors[f];
            L->sub[(size_t)k * n + i] = 1;
            f = L->tors_pfrag[k];
        }
    }

    /* intra pairs: different fragments, bond-graph distance >= 4 */
    int cap = n * (n - 1) / 2 + 1, np = 0;
    L->pairs = malloc(sizeof(int) * 2 * cap);
    for (int i = 0; i < n; ++i) {
        for (int v = 0; v < n; ++v) dist[v] = -1;
        qh = qt = 0; queue[qt++] = i; dist[i] = 0;
        while (qh < qt) {
            int u = queue[qh++];
            for (int v = 0; v < n; ++v)
                if (adj[u * n + v] && dist[v] < 0) { dist[v] = dist[u] + 1; queue[qt++] = v; }
        }
        for (int j = i + 1; j < n; ++j)
            if (L->frag[i] != L->frag[j] && dist[j] >= 4) {
                L->pairs[2 * np] = i; L->pairs[2 * np + 1] = j; ++np;
            }
    }
    L->np = np;

    /* anchor = centroid of the root fragment; radius of gyration of all atoms */
    double c[3] = {0, 0, 0}, ca[3] = {0, 0, 0};
    int nr = 0;
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) ca[a] += ref[3 * i + a];
        if (L->frag[i] == root) { for (int a = 0; a < 3; ++a) c[a] += ref[3 * i + a]; ++nr; }
    }
    for (int a = 0; a < 3; ++a) { L->anchor[a] = c[a] / nr; ca[a] /= n; }
    double s2 = 0.0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) { double d = ref[3 * i + a] - ca[a]; s2 += d * d; }
    L->rg = sqrt(s2 / n);

    free(adj); free(adjr); free(queue); free(dist);
    *out = L;
    return 0;
}

void or_ligand_info(const or_ligand* L, int32_t info[8])
{
    info[0] = L->n; info[1] = L->nf; info[2] = L->nt; info[3] = L->np;
    info[4] = L->root; info[5] = L->depth; info[6] = 0; info[7] = 0;
}
void or_ligand_pairs(const or_ligand* L, int32_t* p)
{
    for (int i = 0; i < 2 * L->np; ++i) p[i] = L->pairs[i];
}
void or_ligand_frag(const or_ligand* L, int32_t* f)
{
    for (int i = 0; i < L->n; ++i) f[i] = L->frag[i];
}
void or_ligand_torsions(const or_ligand* L, int32_t* t)
{
    for (int k = 0; k < L->nt; ++k) {
        t[3 * k] = L->tors_bond[k]; t[3 * k + 1] = L->tors_a[k]; t[3 * k + 2] = L->tors_c[k];
    }
}
double or_ligand_rg(const or_ligand* L) { return L->rg; }
void or_ligand_anchor(const or_ligand* L, double a[3])
{
    a[0] = L->anchor[0]; a[1] = L->anchor[1]; a[2] = L->anchor[2];
}

/* ------------------------------------------------------------------ */
/* Rotations.  Quaternions are (w, x, y, z) = (a, b, c, d) of           */
/* Eq. qvina_eq_1, normalised before use.                               */
/* ------------------------------------------------------------------ */
static void quat_to_mat(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void quat_mul(const double a[4], const double b[4], double o[4])
{
    double r0 = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double r1 = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double r2 = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double r3 = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
}

/* rotation vector -> unit quaternion */
static void rotvec_quat(const double th[3], double q[4])
{
    double a = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    if (a == 0.0) { q[0] = 1; q[1] = q[2] = q[3] = 0; return; }
    double s = sin(0.5 * a) / a;
    q[0] = cos(0.5 * a); q[1] = s * th[0]; q[2] = s * th[1]; q[3] = s * th[2];
}

/* Rodrigues: rotation by psi about unit axis u */
static void axis_angle_mat(const double u[3], double psi, double R[9])
{
    double c = cos(psi), s = sin(psi), t = 1.0 - c;
    R[0] = c + t * u[0] * u[0];        R[1] = t * u[0] * u[1] - s * u[2]; R[2] = t * u[0] * u[2] + s * u[1];
    R[3] = t * u[1] * u[0] + s * u[2]; R[4] = c + t * u[1] * u[1];        R[5] = t * u[1] * u[2] - s * u[0];
    R[6] = t * u[2] * u[0] - s * u[1]; R[7] = t * u[2] * u[1] + s * u[0]; R[8] = c + t * u[2] * u[2];
}

static void matmul3(const double A[9], const double B[9], double C[9])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

static void matvec3(const double A[9], const double v[3], double o[3])
{
    double r0 = A[0] * v[0] + A[1] * v[1] + A[2] * v[2];
    double r1 = A[3] * v[0] + A[4] * v[1] + A[5] * v[2];
    double r2 = A[6] * v[0] + A[7] * v[1] + A[8] * v[2];
    o[0] = r0; o[1] = r1; o[2] = r2;
}

static void cross3(const double a[3], const double b[3], double o[3])
{
    double r0 = a[1] * b[2] - a[2] * b[1];
    double r1 = a[2] * b[0] - a[0] * b[2];
    double r2 = a[0] * b[1] - a[1] * b[0];
    o[0] = r0; o[1] = r1; o[2] = r2;
}

/* ------------------------------------------------------------------ */
/* Forward kinematics (POT -> atom coordinates, Eq. qvina_eq_1).        */
/* Fragment f carries an affine map x = R_f X + b_f of the reference    */
/* coordinates.  Root: R = R(q), b = t - R(q) anchor.  A child joined   */
/* by torsion k composes its parent's map with the rotation by psi_k    */
/* about the reference axis through the child-side atom.               */
/* ------------------------------------------------------------------ */
static void fk_frames(const or_ligand* L, const double* dof, double* Rf, double* bf)
{
    double q[4] = {dof[3], dof[4], dof[5], dof[6]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; ++a) q[a] /= qn;
    double* R0 = Rf + 9 * L->root;
    double* b0 = bf + 3 * L->root;
    quat_to_mat(q, R0);
    double ra[3];
    matvec3(R0, L->anchor, ra);
    for (int a = 0; a < 3; ++a) b0[a] = dof[a] - ra[a];
    for (int idx = 1; idx < L->nf; ++idx) {
        int f = L->frag_bfs[idx];
        int k = L->frag_tors[f];
        int p = L->tors_pfrag[k];
        const double* Xc = L->ref + 3 * L->tors_c[k];
        const double* Xa = L->ref + 3 * L->tors_a[k];
        double u[3] = {Xc[0] - Xa[0], Xc[1] - Xa[1], Xc[2] - Xa[2]};
        double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int a = 0; a < 3; ++a) u[a] /= un;
        double Rk[9];
        axis_angle_mat(u, dof[7 + k], Rk);
        /* local map: X -> Rk (X - Xc) + Xc; composed with the parent's */
        double RkXc[3], loc_b[3], pb[3];
        matvec3(Rk, Xc, RkXc);
        for (int a = 0; a < 3; ++a) loc_b[a] = Xc[a] - RkXc[a];
        matmul3(Rf + 9 * p, Rk, Rf + 9 * f);
        matvec3(Rf + 9 * p, loc_b, pb);
        for (int a = 0; a < 3; ++a) bf[3 * f + a] = pb[a] + bf[3 * p + a];
    }
}

void or_fk(const or_ligand* L, const double* dof, double* xyz)
{
    double* Rf = malloc(sizeof(double) * 9 * L->nf);
    double* bf = malloc(sizeof(double) * 3 * L->nf);
    fk_frames(L, dof, Rf, bf);
    for (int i = 0; i < L->n; ++i) {
        int f = L->frag[i];
        double x[3];
        matvec3(Rf + 9 * f, L->ref + 3 * i, x);
        for (int a = 0; a < 3; ++a) xyz[3 * i + a] = x[a] + bf[3 * f + a];
    }
    free(Rf); free(bf);
}

/* ------------------------------------------------------------------ */
/* Score on given coordinates: E = e_inter + e_intra (Eq. qvina_eq_3)   */
/* and G_i = dE/dx_i.                                                   */
/* ------------------------------------------------------------------ */
int or_score_xyz(const or_ligand* L, const or_grid* G, const double* xyz,
                 double e3[3], double* gxyz, or_flags* fl)
{
    const int n = L->n;
    const size_t msz = (size_t)G->dims[0] * G->dims[1] * G->dims[2];
    double e_inter = 0.0, e_intra = 0.0;
    double min_face = INFINITY, min_cut = INFINITY, min_kink = INFINITY;
    int64_t pin = 0;
    for (int i = 0; i < 3 * n; ++i) gxyz[i] = 0.0;
    for (int i = 0; i < n; ++i) {
        double g[3], fd;
        e_inter += or_trilinear(G->maps + (size_t)L->type[i] * msz, G->dims, G->origin,
                                G->h, G->kappa, xyz + 3 * i, g, &fd);
        for (int a = 0; a < 3; ++a) gxyz[3 * i + a] += g[a];
        if (fd < min_face) min_face = fd;
    }
    for (int p = 0; p < L->np; ++p) {
        int i = L->pairs[2 * p], j = L->pairs[2 * p + 1];
        double dx[3] = {xyz[3 * i] - xyz[3 * j], xyz[3 * i + 1] - xyz[3 * j + 1],
                        xyz[3 * i + 2] - xyz[3 * j + 2]};
        double r = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        if (fabs(r - CUTOFF) < min_cut) min_cut = fabs(r - CUTOFF);
        if (!(r < CUTOFF)) continue;
        ++pin;
        int ti = L->type[i], tj = L->type[j];
        double d = r - T_RADIUS[ti] - T_RADIUS[tj];
        if (pair_is_hyd(ti, tj)) {
            if (fabs(d - 0.5) < min_kink) min_kink = fabs(d - 0.5);
            if (fabs(d - 1.5) < min_kink) min_kink = fabs(d - 1.5);
        }
        if (pair_is_hb(ti, tj)) {
            if (fabs(d + 0.7) < min_kink) min_kink = fabs(d + 0.7);
            if (fabs(d) < min_kink) min_kink = fabs(d);
        }
        double de;
        e_intra += or_pair(ti, tj, r, &de);
        if (r > 0.0)
            for (int a = 0; a < 3; ++a) {
                gxyz[3 * i + a] += de * dx[a] / r;
                gxyz[3 * j + a] -= de * dx[a] / r;
            }
    }
    e3[0] = e_inter + e_intra; e3[1] = e_inter; e3[2] = e_intra;
    if (fl) { fl->min_face = min_face; fl->min_cut = min_cut; fl->min_kink = min_kink; fl->pairs_in = pin; }
    return 0;
}

/* Score and gradient of a POT.  Chain rule through the torsion tree:
 *   dE/dt      = sum_i G_i
 *   torque     = sum_i (x_i - t) x G_i      (world rotation-vector gradient)
 *   dE/dpsi_k  = a_k . sum_{i moved by k} (x_i - x_{c_k}) x G_i
 * with a_k the world axis of torsion k.  For the raw input quaternion p
 * (q = p/|p|):  dE/dp = 2 ((0, torque) (x) q) / |p|. */
int or_score_grad(const or_ligand* L, const or_grid* G, const double* dof,
                  double e3[3], double* grad_dof, double* grad_tan,
                  double* xyz_out, double* gxyz_out, or_flags* fl)
{
    const int n = L->n, nt = L->nt;
    double* xyz = malloc(sizeof(double) * 3 * n);
    double* gx = malloc(sizeof(double) * 3 * n);
    double* Rf = malloc(sizeof(double) * 9 * L->nf);
    double* bf = malloc(sizeof(double) * 3 * L->nf);
    fk_frames(L, dof, Rf, bf);
    for (int i = 0; i < n; ++i) {
        int f = L->frag[i];
        double x[3];
        matvec3(Rf + 9 * f, L->ref + 3 * i, x);
        for (int a = 0; a < 3; ++a) xyz[3 * i + a] = x[a] + bf[3 * f + a];
    }
    or_score_xyz(L, G, xyz, e3, gx, fl);

    double F[3] = {0, 0, 0}, tq[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        double rel[3] = {xyz[3 * i] - dof[0], xyz[3 * i + 1] - dof[1], xyz[3 * i + 2] - dof[2]}, c[3];
        cross3(rel, gx + 3 * i, c);
        for (int a = 0; a < 3; ++a) { F[a] += gx[3 * i + a]; tq[a] += c[a]; }
    }
    double* dpsi = malloc(sizeof(double) * (nt + 1));
    for (int k = 0; k < nt; ++k) {
        const double* Xc = L->ref + 3 * L->tors_c[k];
        const double* Xa = L->ref + 3 * L->tors_a[k];
        double u[3] = {Xc[0] - Xa[0], Xc[1] - Xa[1], Xc[2] - Xa[2]};
        double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int a = 0; a < 3; ++a) u[a] /= un;
        double aw[3];
        matvec3(Rf + 9 * L->tors_pfrag[k], u, aw);
        const double* pc = xyz + 3 * L->tors_c[k];
        double s[3] = {0, 0, 0};
        for (int i = 0; i < n; ++i) {
            if (!L->sub[(size_t)k * n + i]) continue;
            double rel[3] = {xyz[3 * i] - pc[0], xyz[3 * i + 1] - pc[1], xyz[3 * i + 2] - pc[2]}, c[3];
            cross3(rel, gx + 3 * i, c);
            for (int a = 0; a < 3; ++a) s[a] += c[a];
        }
        dpsi[k] = aw[0] * s[0] + aw[1] * s[1] + aw[2] * s[2];
    }
    if (grad_tan) {
        for (int a = 0; a < 3; ++a) { grad_tan[a] = F[a]; grad_tan[3 + a] = tq[a]; }
        for (int k = 0; k < nt; ++k) grad_tan[6 + k] = dpsi[k];
    }
    if (grad_dof) {
        double p[4] = {dof[3], dof[4], dof[5], dof[6]};
        double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        double q[4] = {p[0] / pn, p[1] / pn, p[2] / pn, p[3] / pn};
        double tq4[4] = {0.0, tq[0], tq[1], tq[2]}, gq[4];
        quat_mul(tq4, q, gq);
        for (int a = 0; a < 3; ++a) grad_dof[a] = F[a];
        for (int a = 0; a < 4; ++a) grad_dof[3 + a] = 2.0 * gq[a] / pn;
        for (int k = 0; k < nt; ++k) grad_dof[7 + k] = dpsi[k];
    }
    if (xyz_out) memcpy(xyz_out, xyz, sizeof(double) * 3 * n);
    if (gxyz_out) memcpy(gxyz_out, gx, sizeof(double) * 3 * n);
    free(xyz); free(gx); free(Rf); free(bf); free(dpsi);
    return 0;
}

/* e_inter straight from receptor atom pairs (no grid), for the
 * grid-versus-pairwise check. */
double or_inter_pairwise(int n_rec, const float* rec, const int32_t* rtype,
                         int n, const double* xyz, const int32_t* type)
{
    double e = 0.0;
    for (int i = 0; i < n; ++i)
        for (int r = 0; r < n_rec; ++r) {
            double dx = xyz[3 * i] - rec[3 * r], dy = xyz[3 * i + 1] - rec[3 * r + 1],
                   dz = xyz[3 * i + 2] - rec[3 * r + 2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (d < CUTOFF) e += or_pair(type[i], rtype[r], d, NULL);
        }
    return e;
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two */
/* 64x64->128 multiplies; the key is bumped by the Weyl constants       */
/* between rounds.                                                      */
/* ------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t h0, l0, h1, l1;
        mulhilo64(M0, c0, &h0, &l0);
        mulhilo64(M1, c2, &h1, &l1);
        uint64_t n0 = h1 ^ c1 ^ k0, n1 = l1, n2 = h0 ^ c3 ^ k1, n3 = l0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draws of one chain: counter = (block, step, chain, job), key = (seed, 0).
 * step 0 is the initial pose; MC step s uses step s + 1.  Uniform in
 * [0, 1): the top 24 bits of a word times 2^-24 (exact in binary32). */
static void draw_block(uint64_t seed, int job, int chain, uint64_t step, uint64_t block,
                       uint64_t w[4])
{
    uint64_t ctr[4] = {block, step, (uint64_t)chain, (uint64_t)job};
    uint64_t key[2] = {seed, 0};
    or_philox4x64_10(ctr, key, w);
}
static double u01(uint64_t w) { return (double)(w >> 40) * (1.0 / 16777216.0); }

/* ------------------------------------------------------------------ */
/* RILC-BFGS in the 6+T tangent space (Eqs. qvina_eq_6 .. qvina_eq_12). */
/* Readings: the POT update of Eq. qvina_eq_9 is additive on t and psi  */
/* and a left rotation q <- exp(lambda d_theta) q on the orientation;   */
/* the Armijo / weak-Wolfe inequalities as printed are the shrink and   */
/* grow branches of the Lewis-Overton bisection, a trial is accepted    */
/* when it satisfies both; H0 = (s.y / y.y) I from the newest pair;     */
/* separate epsilons for the curvature test and the termination test;   */
/* if no trial is accepted the step falls back to the last point that   */
/* passed Armijo, else the run stops.                                   */
/* ------------------------------------------------------------------ */
static void retract(int nt, const double* x, const double* d, double lam, double* o)
{
    for (int a = 0; a < 3; ++a) o[a] = x[a] + lam * d[a];
    double th[3] = {lam * d[3], lam * d[4], lam * d[5]}, dq[4], q[4];
    rotvec_quat(th, dq);
    quat_mul(dq, x + 3, q);
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; ++a) o[3 + a] = q[a] / qn;
    for (int k = 0; k < nt; ++k) o[7 + k] = x[7 + k] + lam * d[6 + k];
}

/* x (+) lam d as BFGS moves a pose (7 + nt values) along a tangent
 * direction d (6 + nt values); exported for the tests of its convention. */
void or_retract(int nt, const double* x, const double* d, double lam, double* o) { retract(nt, x, d, lam, o); }

static double dot(int n, const double* a, const double* b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* One problem for the BFGS core: an objective with gradient in an nd-dim
 * tangent space and a retraction x (+) lambda d on nx-dim points. */
typedef struct {
    void (*eval)(void* ctx, const double* x, double* f, double* g);
    void (*retract)(void* ctx, const double* x, const double* d, double lam, double* o);
    void* ctx;
    int nx, nd;
} bfgs_problem;

/* How close a run came to deciding otherwise (see or_bfgs_margins). */
static void margin_min(double* m, double v) { if (m && v < *m) *m = v; }

static int bfgs_core(const bfgs_problem* pb, const or_bfgs_params* P, const double* x0,
                     double* xout, double* fout, int64_t* n_evals, int32_t* n_iters,
                     or_bfgs_margins* mg)
{
    if (mg) { mg->armijo = mg->wolfe = mg->curvature = mg->descent = INFINITY; }
    const int nd = pb->nd, nx = pb->nx, m = P->m > 0 ? P->m : 1;
    double *x = malloc(sizeof(double) * nx), *xt = malloc(sizeof(double) * nx),
           *xa = malloc(sizeof(double) * nx);
    double *g = malloc(sizeof(double) * nd), *gt = malloc(sizeof(double) * nd),
           *ga = malloc(sizeof(double) * nd), *d = malloc(sizeof(double) * nd),
           *qv = malloc(sizeof(double) * nd);
    double *S = malloc(sizeof(double) * m * nd), *Y = malloc(sizeof(double) * m * nd);
    double *rh = malloc(sizeof(double) * m), *al = malloc(sizeof(double) * m);
    int hn = 0; /* pairs held; pair 0 is the oldest */
    int64_t ne = 0;
    int it = 0;
    double f, ft = 0.0, fa = 0.0;
    memcpy(x, x0, sizeof(double) * nx);
    pb->eval(pb->ctx, x, &f, g); ++ne;
    for (it = 0; it < P->max_iter; ++it) {
        double gn = sqrt(dot(nd, g, g));
        if (gn <= P->eps_g) break;                 /* Eq. qvina_eq_12 */
        /* two-loop recursion over the held pairs: d = -H g (Eq. qvina_eq_6 when empty) */
        for (int i = 0; i < nd; ++i) qv[i] = g[i];
        for (int h = hn - 1; h >= 0; --h) {
            al[h] = rh[h] * dot(nd, S + h * nd, qv);
            for (int i = 0; i < nd; ++i) qv[i] -= al[h] * Y[h * nd + i];
        }
        if (hn > 0) {
            double gam = dot(nd, S + (hn - 1) * nd, Y + (hn - 1) * nd) /
                         dot(nd, Y + (hn - 1) * nd, Y + (hn - 1) * nd);
            for (int i = 0; i < nd; ++i) qv[i] *= gam;
        }
        for (int h = 0; h < hn; ++h) {
            double b = rh[h] * dot(nd, Y + h * nd, qv);
            for (int i = 0; i < nd; ++i) qv[i] += S[h * nd + i] * (al[h] - b);
        }
        for (int i = 0; i < nd; ++i) d[i] = -qv[i];
        double gd = dot(nd, g, d);
        double d1 = 0.0;
        for (int i = 0; i < nd; ++i) d1 += fabs(d[i]);
        margin_min(mg ? &mg->descent : NULL, fabs(gd) / (1e-300 + d1 * (1.0 + gn)));
        if (!(gd < 0.0)) break;                    /* not a descent direction */
        /* Lewis-Overton bisection (Eqs. qvina_eq_7 and qvina_eq_8) */
        double a_lo = 0.0, lam = 1.0, lam_ok = -1.0, beta = 0.0;
        int beta_inf = 1, accepted = 0;
        for (int tr = 0; tr < P->ls_max; ++tr) {
            pb->retract(pb->ctx, x, d, lam, xt);
            pb->eval(pb->ctx, xt, &ft, gt); ++ne;
            if (mg) {
                double gmax = 0.0;
                for (int i = 0; i < nd; ++i) gmax = fmax(gmax, fabs(gt[i]));
                margin_min(&mg->armijo, fabs(ft - (f + P->rho * lam * gd)) / (1.0 + fabs(ft)));
                if (!(ft > f + P->rho * lam * gd))
                    margin_min(&mg->wolfe, fabs(dot(nd, gt, d) - P->sigma * gd) / (1e-300 + d1 * (1.0 + gmax)));
            }
            if (ft > f + P->rho * lam * gd) {          /* Armijo fails: shrink */
                beta = lam; beta_inf = 0;
            } else if (dot(nd, gt, d) < P->sigma * gd) { /* Wolfe fails: grow */
                a_lo = lam;
                memcpy(xa, xt, sizeof(double) * nx); memcpy(ga, gt, sizeof(double) * nd); fa = ft;
            } else {
                accepted = 1; lam_ok = lam; break;
            }
            lam = beta_inf ? 2.0 * lam : 0.5 * (a_lo + beta);
        }
        if (!accepted) {
            if (a_lo > 0.0) {
                lam_ok = a_lo;
                memcpy(xt, xa, sizeof(double) * nx); memcpy(gt, ga, sizeof(double) * nd); ft = fa;
            } else {
                break;
            }
        }
        /* s = lambda d, y = g+ - g (Eq. qvina_eq_10); cautious update (Eq. qvina_eq_11) */
        double* sv = qv; /* qv and ga are free again: reuse them for s and y */
        double* yv = ga;
        for (int i = 0; i < nd; ++i) { sv[i] = lam_ok * d[i]; yv[i] = gt[i] - g[i]; }
        double ys = dot(nd, yv, sv), ss = dot(nd, sv, sv);
        margin_min(mg ? &mg->curvature : NULL, fabs(ys / ss - P->eps_c * gn) / (1e-300 + fabs(ys / ss) + P->eps_c * gn));
        if (ys / ss > P->eps_c * gn) {
            if (hn == m) { /* drop the oldest */
                memmove(S, S + nd, sizeof(double) * (m - 1) * nd);
                memmove(Y, Y + nd, sizeof(double) * (m - 1) * nd);
                memmove(rh, rh + 1, sizeof(double) * (m - 1));
                --hn;
            }
            memcpy(S + hn * nd, sv, sizeof(double) * nd);
            memcpy(Y + hn * nd, yv, sizeof(double) * nd);
            rh[hn] = 1.0 / ys;
            ++hn;
        }
        memcpy(x, xt, sizeof(double) * nx);        /* Eq. qvina_eq_9 */
        memcpy(g, gt, sizeof(double) * nd);
        f = ft;
    }
    memcpy(xout, x, sizeof(double) * nx);
    *fout = f;
    if (n_evals) *n_evals = ne;
    if (n_iters) *n_iters = it;
    free(x); free(xt); free(xa); free(g); free(gt); free(ga); free(d); free(qv);
    free(S); free(Y); free(rh); free(al);
    return 0;
}

typedef struct { const or_ligand* L; const or_grid* G; double* min_flag; } pose_ctx;

static void pose_eval(void* c, const double* x, double* f, double* g)
{
    const pose_ctx* pc = (const pose_ctx*)c;
    double e3[3];
    or_flags fl;
    or_score_grad(pc->L, pc->G, x, e3, NULL, g, NULL, NULL, pc->min_flag ? &fl : NULL);
    if (pc->min_flag) margin_min(pc->min_flag, fmin(fl.min_face, fmin(fl.min_cut, fl.min_kink)));
    *f = e3[0];
}

static void pose_retract(void* c, const double* x, const double* d, double lam, double* o)
{
    retract(((const pose_ctx*)c)->L->nt, x, d, lam, o);
}

int or_bfgs(const or_ligand* L, const or_grid* G, const or_bfgs_params* P,
            const double* x0, double* xout, double* fout, int64_t* n_evals, int32_t* n_iters)
{
    pose_ctx pc = {L, G, NULL};
    bfgs_problem pb = {pose_eval, pose_retract, &pc, 7 + L->nt, 6 + L->nt};
    return bfgs_core(&pb, P, x0, xout, fout, n_evals, n_iters, NULL);
}

int or_bfgs_margins_run(const or_ligand* L, const or_grid* G, const or_bfgs_params* P,
                        const double* x0, double* xout, double* fout, int64_t* n_evals,
                        int32_t* n_iters, or_bfgs_margins* mg)
{
    pose_ctx pc = {L, G, &mg->pose};
    mg->pose = INFINITY;
    bfgs_problem pb = {pose_eval, pose_retract, &pc, 7 + L->nt, 6 + L->nt};
    return bfgs_core(&pb, P, x0, xout, fout, n_evals, n_iters, mg);
}

typedef struct { or_eval_fn fn; void* user; } flat_ctx;

static void flat_eval(void* c, const double* x, double* f, double* g)
{
    const flat_ctx* fc = (const flat_ctx*)c;
    fc->fn(fc->user, x, f, g);
}

typedef struct { flat_ctx fc; int n; } flat_ctx_n;

static void flat_retract_n(void* c, const double* x, const double* d, double lam, double* o)
{
    const flat_ctx_n* f = (const flat_ctx_n*)c;
    for (int i = 0; i < f->n; ++i) o[i] = x[i] + lam * d[i];
}

static void flat_eval_n(void* c, const double* x, double* f, double* g)
{
    flat_eval(&((flat_ctx_n*)c)->fc, x, f, g);
}

int or_bfgs_generic(int n, or_eval_fn fn, void* user, const or_bfgs_params* P,
                    const double* x0, double* xout, double* fout, int64_t* n_evals,
                    int32_t* n_iters)
{
    flat_ctx_n c = {{fn, user}, n};
    bfgs_problem pb = {flat_eval_n, flat_retract_n, &c, n, n};
    return bfgs_core(&pb, P, x0, xout, fout, n_evals, n_iters, NULL);
}

/* ------------------------------------------------------------------ */
/* Monte Carlo chain (Supplementary Algorithm 2, per thread).           */
/* Initial pose (not optimised): t uniform in the lattice box, q        */
/* uniform on S^3 (Shoemake), psi uniform in [-pi, pi).                 */
/* Mutation (Eq. qvina_eq_2): one entity chosen uniformly among         */
/* {position, orientation, psi_1..psi_T}; position moves by a uniform   */
/* point of a ball of radius mut_pos_amp; orientation turns by a        */
/* uniform rotation vector of a ball of radius mut_rot_amp / R_g; a     */
/* torsion is redrawn uniformly.                                        */
/* Step: mutate -> BFGS -> Metropolis with P = exp((e_cur - e_o)/T)     */
/* for e_o >= e_cur (Eq. qvina_eq_13 read with the 1.2 as a divisor of  */
/* the exponent) -> a candidate better than the best is refined by a    */
/* second BFGS and becomes both best and current.                      */
/* ------------------------------------------------------------------ */
int or_init_pose(const or_ligand* L, const or_grid* G, uint64_t seed, int job, int chain,
                 double* dof)
{
    const int nt = L->nt, nu = 6 + nt;
    double u[6 + 64];
    for (int b = 0; 4 * b < nu; ++b) {
        uint64_t w[4];
        draw_block(seed, job, chain, 0, (uint64_t)b, w);
        for (int c = 0; c < 4 && 4 * b + c < nu; ++c) u[4 * b + c] = u01(w[c]);
    }
    for (int a = 0; a < 3; ++a) {
        double lo = (double)G->origin[a], ext = (double)G->h * (G->dims[a] - 1);
        dof[a] = lo + u[a] * ext;
    }
    double s1 = sqrt(1.0 - u[3]), s2 = sqrt(u[3]);
    double a1 = 2.0 * PI * u[4], a2 = 2.0 * PI * u[5];
    dof[3] = s2 * cos(a2);
    dof[4] = s1 * sin(a1);
    dof[5] = s1 * cos(a1);
    dof[6] = s2 * sin(a2);
    for (int k = 0; k < nt; ++k) dof[7 + k] = -PI + 2.0 * PI * u[6 + k];
    return 0;
}

static void mutate(const or_ligand* L, const or_mc_params* P, const uint64_t w[8], double* x)
{
    const int nt = L->nt;
    uint64_t n_ent = (uint64_t)(2 + nt);
    int ent = (int)(((w[0] >> 32) * n_ent) >> 32);
    double u1 = u01(w[1]), u2 = u01(w[2]), u3 = u01(w[3]), u4 = u01(w[4]);
    double ur = u01(w[5]), ua = u01(w[6]);
    double r12 = sqrt(-2.0 * log(1.0 - u1)), r34 = sqrt(-2.0 * log(1.0 - u3));
    double v[3] = {r12 * cos(2.0 * PI * u2), r12 * sin(2.0 * PI * u2), r34 * cos(2.0 * PI * u4)};
    double vn2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double dir[3] = {0.0, 0.0, 1.0};
    if (vn2 > 0.0) { double vn = sqrt(vn2); dir[0] = v[0] / vn; dir[1] = v[1] / vn; dir[2] = v[2] / vn; }
    double rad = cbrt(ur);
    if (ent == 0) {
        for (int a = 0; a < 3; ++a) x[a] += P->mut_pos_amp * rad * dir[a];
    } else if (ent == 1) {
        double amp = P->mut_rot_amp / fmax(L->rg, 1e-3) * rad;
        double th[3] = {amp * dir[0], amp * dir[1], amp * dir[2]}, dq[4], q[4];
        rotvec_quat(th, dq);
        quat_mul(dq, x + 3, q);
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int a = 0; a < 4; ++a) x[3 + a] = q[a] / qn;
    } else {
        x[7 + (ent - 2)] = -PI + 2.0 * PI * ua;
    }
}

/* One mutation (Eq. qvina_eq_2 with the readings above) of the pose x
 * (7 + nt values, changed in place) from the step's 8 Philox words w; for the
 * tests of its distributions. */
void or_mutate(const or_ligand* L, const or_mc_params* P, const uint64_t w[8], double* x) { mutate(L, P, w, x); }

/* ---- first-order consistency check ------------------------------------
 * Eqs. qvina_eq_4 and qvina_eq_5 and the check of Supplementary Algorithm
 * 2.  Readings: the neighbouring conformation of the mutated pose is the
 * chain's current pose, the one it was mutated from, with the gradient of
 * its last evaluation; the coordinates p tested are those the mutation
 * moved (the translation, the rotation vector, or the one torsion).  The
 * check passes, and BFGS runs, when in some moved coordinate the derivative
 * changes sign between the two poses (Eq. qvina_eq_4) or disagrees with the
 * secant slope from the current pose (Eq. qvina_eq_5).  Otherwise the
 * mutated pose lies on the slope it came up from in every moved direction,
 * a descent from it would return towards the current basin, and the step
 * ends without optimisation or Metropolis move. */
static int sgn(double v) { return (v > 0.0) - (v < 0.0); }

int or_consistency_passes(int nt, const double* x, double fx, const double* gx,
                          const double* y, double fy, const double* gy, int p_lo, int p_hi)
{
    double dlt[6 + 32];
    for (int a = 0; a < 3; ++a) dlt[a] = x[a] - y[a];
    /* rotation vector of q_x conj(q_y), w >= 0 */
    double qx[4], qy[4];
    const double nx = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6]);
    const double ny = sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6]);
    for (int a = 0; a < 4; ++a) { qx[a] = x[3 + a] / nx; qy[a] = y[3 + a] / ny; }
    const double cy[4] = {qy[0], -qy[1], -qy[2], -qy[3]};
    double qd[4];
    quat_mul(qx, cy, qd);
    if (qd[0] < 0.0) for (int a = 0; a < 4; ++a) qd[a] = -qd[a];
    const double vn = sqrt(qd[1] * qd[1] + qd[2] * qd[2] + qd[3] * qd[3]);
    const double ang = 2.0 * atan2(vn, qd[0]);
    for (int a = 0; a < 3; ++a) dlt[3 + a] = vn > 0.0 ? ang * qd[1 + a] / vn : 0.0;
    for (int k = 0; k < nt; ++k) {
        double d = x[7 + k] - y[7 + k];
        d -= 2.0 * PI * floor((d + PI) / (2.0 * PI));   /* into [-pi, pi) */
        if (d == -PI) d = PI;                          /* (-pi, pi] */
        dlt[6 + k] = d;
    }
    for (int p = p_lo; p < p_hi; ++p) {
        const int sx = sgn(gx[p]);
        if (sx * sgn(gy[p]) <= 0) return 1;                    /* Eq. qvina_eq_4 */
        if (sx * sgn(fx - fy) * sgn(dlt[p]) <= 0) return 1;    /* Eq. qvina_eq_5 */
    }
    return 0;
}

/* Eq. qvina_eq_13 (reading 13): the candidate e_o replaces the current e_i
 * when it is lower, or when the step's uniform u = u01(word) is below
 * exp((e_i - e_o) / T).  The chain's decision; exported for its tests. */
int or_metropolis_accepts(double e_cur, double e_o, uint64_t word, double temperature)
{
    return e_o < e_cur || u01(word) < exp((e_cur - e_o) / temperature);
}

int or_mc_chain(const or_ligand* L, const or_grid* G, const or_mc_params* P,
                int job, int chain, double* best_dof, double* best_e, int64_t* n_evals)
{
    const int nx = 7 + L->nt;
    double *cur = malloc(sizeof(double) * nx), *mut = malloc(sizeof(double) * nx),
           *opt = malloc(sizeof(double) * nx), *ref = malloc(sizeof(double) * nx),
           *gt = malloc(sizeof(double) * (nx));
    int64_t ne = 0, e1;
    int32_t it;
    or_init_pose(L, G, P->seed, job, chain, cur);
    double e_cur;
    pose_ctx pc = {L, G, NULL};
    pose_eval(&pc, cur, &e_cur, gt); ++ne;
    double e_best = e_cur;
    memcpy(best_dof, cur, sizeof(double) * nx);
    or_bfgs_params rp = P->bfgs;
    rp.max_iter = P->refine_max_iter;
    const int nd = 6 + L->nt;
    double* gm = malloc(sizeof(double) * nd);
    /* gt holds the gradient at the current pose (the check's neighbour) */
    for (int s = 0; s < P->steps; ++s) {
        uint64_t w[8];
        draw_block(P->seed, job, chain, (uint64_t)s + 1, 0, w);
        draw_block(P->seed, job, chain, (uint64_t)s + 1, 1, w + 4);
        memcpy(mut, cur, sizeof(double) * nx);
        mutate(L, P, w, mut);
        if (P->consistency) {
            /* the check evaluates the mutated pose; when BFGS follows, this is
             * its first evaluation (counted there) */
            const int ent = (int)(((w[0] >> 32) * (uint64_t)(2 + L->nt)) >> 32);
            const int p_lo = ent == 0 ? 0 : (ent == 1 ? 3 : 4 + ent);
            const int p_hi = ent <= 1 ? p_lo + 3 : p_lo + 1;
            double fm;
            pose_eval(&pc, mut, &fm, gm);
            if (!or_consistency_passes(L->nt, mut, fm, gm, cur, e_cur, gt, p_lo, p_hi)) { ++ne; continue; }
        }
        double e_o;
        or_bfgs(L, G, &P->bfgs, mut, opt, &e_o, &e1, &it); ne += e1;
        int moved = 0;
        if (or_metropolis_accepts(e_cur, e_o, w[7], P->temperature)) {
            memcpy(cur, opt, sizeof(double) * nx); e_cur = e_o;
            moved = 1;
        }
        if (e_o < e_best) {
            double e_r;
            or_bfgs(L, G, &rp, opt, ref, &e_r, &e1, &it); ne += e1;
            memcpy(best_dof, ref, sizeof(double) * nx); e_best = e_r;
            memcpy(cur, ref, sizeof(double) * nx); e_cur = e_r;
            moved = 1;
        }
        if (moved && P->consistency) {
            /* the neighbour's gradient (an oracle-side re-evaluation; the
             * kernel keeps the one its BFGS ended with, so it is not counted) */
            double f;
            pose_eval(&pc, cur, &f, gt);
        }
    }
    *best_e = e_best;
    if (n_evals) *n_evals = ne;
    free(cur); free(mut); free(opt); free(ref); free(gt);
    free(gm);
    return 0;
}

int or_dock(int n_lig, or_ligand* const* ligs, int n_grids, const or_grid* grids,
            int n_jobs, const int32_t* jobs, const or_mc_params* P, int stride,
            int n_threads, double* cbe, double* cbd, int64_t* cev, double* jbe, int32_t* jbc)
{
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[2 * j] < 0 || jobs[2 * j] >= n_lig || jobs[2 * j + 1] < 0 ||
            jobs[2 * j + 1] >= n_grids) return -1;
        if (7 + ligs[jobs[2 * j]]->nt > stride) return -1;
    }
    const int64_t total = (int64_t)n_jobs * P->chains;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t w = 0; w < total; ++w) {
        int j = (int)(w / P->chains), c = (int)(w % P->chains);
        const or_ligand* L = ligs[jobs[2 * j]];
        double* bd = cbd + (size_t)w * stride;
        for (int i = 0; i < stride; ++i) bd[i] = 0.0;
        or_mc_chain(L, &grids[jobs[2 * j + 1]], P, j, c, bd, cbe + w, cev + w);
    }
    for (int j = 0; j < n_jobs; ++j) {
        int bc = 0;
        for (int c = 1; c < P->chains; ++c)
            if (cbe[(size_t)j * P->chains + c] < cbe[(size_t)j * P->chains + bc]) bc = c;
        jbc[j] = bc;
        jbe[j] = cbe[(size_t)j * P->chains + bc];
    }
    return 0;
}

/* ---- output stage ------------------------------------------------------
 * Methods (end of "Accelerated Docking with QuickVina 2-GPU 2.1") and the
 * last steps of Supplementary Algorithm 2: every chain reports its best
 * pose; the collected poses are clustered and sorted; the selected ones are
 * refined and rescored; then an r.m.s.d. filter and a final sort give the
 * top k.  Readings of what the paper leaves open:
 *  - order: ascending energy, ties to the lower chain index (NaN last);
 *  - clustering: walking that order, a pose is kept unless its heavy-atom
 *    r.m.s.d. (same atom order, no symmetry) to an already kept pose is
 *    below rmsd_cut; at most `modes` are kept;
 *  - refinement: BFGS from each kept pose with refine_max_iter iterations
 *    (the receptor is rigid, so there is no pocket refinement);
 *  - rescoring: the refined pose's E = e_inter + e_intra is the sort key,
 *    and the reported affinity is e_inter / (1 + affinity_w T);
 *  - filter and final sort: ascending rescored energy, ties to the earlier
 *    kept pose; a pose within rmsd_cut of a better one is dropped. */
static int precedes(double ea, int ia, double eb, int ib)
{
    /* a before b: smaller energy, NaN after every number, then lower index */
    const int na = ea != ea, nb = eb != eb;
    if (na != nb) return nb;
    if (!na && ea != eb) return ea < eb;
    return ia < ib;
}

static double rmsd(int n, const double* a, const double* b)
{
    double s = 0.0;
    for (int i = 0; i < 3 * n; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
    return sqrt(s / n);
}

int or_output_stage(const or_ligand* L, const or_grid* G, int n_chains, const double* dof,
                    const double* e, const or_output_params* P, int32_t* n_out,
                    int32_t* out_chain, double* out_e, double* out_aff, double* out_dof,
                    double margins[2])
{
    if (n_chains < 0 || P->modes < 1 || !(P->rmsd_cut >= 0.0)) return -1;
    const int n = L->n, nd = 7 + L->nt, k = P->modes;
    double m_rmsd = INFINITY, m_gap = INFINITY;
    /* 1. sort the chains (insertion sort on (energy, index)) */
    int* order = malloc(sizeof(int) * (n_chains > 0 ? n_chains : 1));
    for (int c = 0; c < n_chains; ++c) {
        int p = c;
        while (p > 0 && precedes(e[c], c, e[order[p - 1]], order[p - 1])) {
            order[p] = order[p - 1];
            --p;
        }
        order[p] = c;
    }
    /* 2. greedy r.m.s.d. clustering over that order */
    double* kx = malloc(sizeof(double) * 3 * n * k);
    int* kc = malloc(sizeof(int) * k);
    double* x = malloc(sizeof(double) * 3 * n);
    int nk = 0;
    for (int r = 0; r < n_chains && nk < k; ++r) {
        const int c = order[r];
        or_fk(L, dof + (size_t)c * nd, x);
        int keep = 1;
        for (int q = 0; q < nk; ++q) {
            const double d = rmsd(n, x, kx + (size_t)3 * n * q);
            if (fabs(d - P->rmsd_cut) < m_rmsd) m_rmsd = fabs(d - P->rmsd_cut);
            if (d < P->rmsd_cut) { keep = 0; break; }
        }
        if (!keep) continue;
        memcpy(kx + (size_t)3 * n * nk, x, sizeof(double) * 3 * n);
        kc[nk++] = c;
    }
    /* 3. refine and rescore each kept pose */
    double* rx = malloc(sizeof(double) * (size_t)nd * (nk > 0 ? nk : 1));
    double* re = malloc(sizeof(double) * (nk > 0 ? nk : 1));
    double* ra = malloc(sizeof(double) * (nk > 0 ? nk : 1));
    for (int q = 0; q < nk; ++q) {
        double* xo = rx + (size_t)nd * q;
        const double* x0 = dof + (size_t)kc[q] * nd;
        if (P->refine_max_iter > 0) {
            or_bfgs_params bp = P->bfgs;
            bp.max_iter = P->refine_max_iter;
            double f;
            int64_t ne;
            int32_t ni;
            or_bfgs(L, G, &bp, x0, xo, &f, &ne, &ni);
        } else {
            memcpy(xo, x0, sizeof(double) * nd);
        }
        const double qn = sqrt(xo[3] * xo[3] + xo[4] * xo[4] + xo[5] * xo[5] + xo[6] * xo[6]);
        for (int a = 3; a < 7; ++a) xo[a] /= qn;
        double e3[3];
        or_score_grad(L, G, xo, e3, NULL, NULL, kx + (size_t)3 * n * q, NULL, NULL);
        re[q] = e3[0];
        ra[q] = e3[1] / (1.0 + P->affinity_w * L->nt);
    }
    /* 4. final sort of the refined poses and r.m.s.d. filter */
    int* fo = malloc(sizeof(int) * (nk > 0 ? nk : 1));
    for (int q = 0; q < nk; ++q) {
        int p = q;
        while (p > 0 && precedes(re[q], q, re[fo[p - 1]], fo[p - 1])) {
            fo[p] = fo[p - 1];
            --p;
        }
        fo[p] = q;
    }
    for (int q = 1; q < nk; ++q) {
        const double g = fabs(re[fo[q]] - re[fo[q - 1]]);
        if (g < m_gap) m_gap = g;
    }
    int no = 0;
    for (int r = 0; r < nk; ++r) {
        const int q = fo[r];
        int keep = 1;
        for (int s = 0; s < no; ++s) {
            int qs = -1;
            for (int t = 0; t < nk; ++t)
                if (kc[t] == out_chain[s]) qs = t;
            const double d = rmsd(n, kx + (size_t)3 * n * q, kx + (size_t)3 * n * qs);
            if (fabs(d - P->rmsd_cut) < m_rmsd) m_rmsd = fabs(d - P->rmsd_cut);
            if (d < P->rmsd_cut) { keep = 0; break; }
        }
        if (!keep) continue;
        out_chain[no] = kc[q];
        out_e[no] = re[q];
        out_aff[no] = ra[q];
        memcpy(out_dof + (size_t)nd * no, rx + (size_t)nd * q, sizeof(double) * nd);
        ++no;
    }
    *n_out = no;
    if (margins) { margins[0] = m_rmsd; margins[1] = m_gap; }
    free(order); free(kx); free(kc); free(x); free(rx); free(re); free(ra); free(fo);
    return 0;
}

/* ---- receptor surface points and point features --------------------------
 * Methods, "Pocket prediction with P2Rank": points on the solvent-accessible
 * surface, and per point a distance-weighted sum of atomic properties over
 * the atoms within 6 A (Eq. prank_eq_1) plus the protrusion count of atoms
 * within 10 A.  Readings: the atom radius is the X-Score radius of its XS
 * type plus the probe; the surface is sampled along given unit directions;
 * the properties are the one-hot XS type and its hydrophobic, donor and
 * acceptor flags.  Every in/out decision is taken on binary32 values with
 * explicit fused multiply-adds, as stated in the header; sums are binary64. */
static float sas_radius(int t, float probe) { return (float)T_RADIUS[t] + probe; }

int or_sas_points(int n_rec, const float* x, const int32_t* type, int n_dirs, const float* dirs, float probe,
                  int cap, float* pts, int32_t* atom)
{
    if (n_rec < 0 || n_dirs < 0 || !(probe >= 0.0f)) return -1;
    for (int a = 0; a < n_rec; ++a)
        if (type[a] < 0 || type[a] >= OR_NTYPES) return -1;
    int n = 0;
    for (int a = 0; a < n_rec; ++a) {
        const float ra = sas_radius(type[a], probe);
        for (int k = 0; k < n_dirs; ++k) {
            float c[3];
            for (int d = 0; d < 3; ++d) c[d] = fmaf(ra, dirs[3 * k + d], x[3 * a + d]);
            int buried = 0;
            for (int b = 0; b < n_rec && !buried; ++b) {
                if (b == a) continue;
                const float rb = sas_radius(type[b], probe);
                const float dx = c[0] - x[3 * b], dy = c[1] - x[3 * b + 1], dz = c[2] - x[3 * b + 2];
                const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                if (d2 < rb * rb) buried = 1;
            }
            if (buried) continue;
            if (n < cap) {
                for (int d = 0; d < 3; ++d) pts[3 * n + d] = c[d];
                atom[n] = a;
            }
            ++n;
        }
    }
    return n;
}

void or_point_features(int n_rec, const float* x, const int32_t* type, int n_pts, const float* pts, double* feat)
{
    for (int p = 0; p < n_pts; ++p) {
        double* f = feat + (size_t)12 * p;
        for (int c = 0; c < 12; ++c) f[c] = 0.0;
        for (int b = 0; b < n_rec; ++b) {
            const float dx = pts[3 * p] - x[3 * b], dy = pts[3 * p + 1] - x[3 * b + 1], dz = pts[3 * p + 2] - x[3 * b + 2];
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            if (d2 < 100.0f) f[11] += 1.0;
            if (!(d2 < 36.0f)) continue;
            const double w = 1.0 - sqrt((double)d2) / 6.0;     /* Eq. prank_eq_1 weight */
            const int t = type[b];
            f[t] += w;
            if (T_HYD[t]) f[8] += w;
            if (T_DON[t]) f[9] += w;
            if (T_ACC[t]) f[10] += w;
        }
    }
}
