// pv_api.cpp -- the C ABI of include/pvdock.h: argument checks, device
// tables of grids, ligands and dock plans, and the launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pvdock.h"
#include "pv_internal.h"

using namespace pv;

namespace {

thread_local std::string g_err;

pv_status fail(pv_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

pv_status hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PV_E_NOMEM : PV_E_DEVICE;
}

#define HIP_TRY(expr, what)                                 \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return hip_fail(_e, what);    \
    } while (0)

template <class T>
pv_status upload(T** dst, const T* src, size_t n, const char* what)
{
    *dst = nullptr;
    if (n == 0) n = 1;  // keep a valid pointer for empty tables
    hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, what);
    if (src) {
        e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) { (void)hipFree(*dst); *dst = nullptr; return hip_fail(e, what); }
    }
    return PV_OK;
}

void dfree(void* p)
{
    if (p) (void)hipFree(p);
}

}  // namespace

// One autotuner choice: the key of a size class's launch, and its schedule.
struct TuneEntry {
    int32_t max_atoms, max_pairs, max_ell, max_tors;
    int64_t items;
    int32_t steps, max_iter, refine_max_iter, m, ls_max, consistency;
    int32_t variant, workgroups;
};

constexpr size_t kTuneMemory = 256;   // autotuner choices a context remembers
constexpr int64_t kTuneFill = 8;      // a tuning run's chains: this many times the widest candidate's workgroups

struct pv_ctx {
    int device;
    int n_cu;
    int lds_per_block;   // dynamic LDS bytes one workgroup may use
    uint32_t magic;
    void* scratch;             // the device's allocation-free scratch (device address), or NULL
    hipError_t scratch_err;    // why it is NULL
    std::mutex tune_mu;
    std::vector<TuneEntry> tune;
};

struct pv_grids {
    pv_ctx* ctx;
    int32_t n_boxes;
    float kappa;
    float* maps;
    int32_t* dims;
    float* geom;
    int64_t* map_off;
    float4* atoms;
    int32_t* atom_off;
    int32_t* tile_off;
    int64_t n_tiles;
    std::vector<int32_t> h_dims;
    std::vector<float> h_geom;
    std::vector<int64_t> h_off;
};

struct pv_ligands {
    pv_ctx* ctx;
    int32_t n_lig;
    int32_t max_atoms, max_pairs, max_tors;
    DevLig* ligs;
    float4* atoms;
    int16_t* perm;
    DevFrag* frags;
    int8_t* tors_frag;
    uint32_t* pairs;
    uint32_t* ell;
    uint32_t* pslot;
    int32_t max_ell;
    std::vector<std::array<int32_t, 9>>* info;   // pv_ligands_info's 8 values, then the slot-table size
};

struct DockGroup {
    LigDev lv;               // the ligand view with this group's maxima
    LaunchShape shape;       // batched launch over the group's (job, chain) items
    LaunchShape plain_shape; // one launch per job of the group
    int32_t workgroups;
    int32_t n_jobs;
    int32_t* job_map;        // device [n_jobs]: group job -> plan job
};

struct pv_plan {
    pv_ctx* ctx;
    const pv_grids* grids;
    const pv_ligands* ligs;
    SearchParams sp;
    int32_t n_jobs;
    int2* jobs;
    std::vector<int2> h_jobs;
    uint32_t* queue;
    float* scratch_best;      // chain_best_e when the caller does not want it
    int64_t* scratch_evals;   // chain_evals when only job_evals is wanted
    int32_t* scratch_status;  // chain_status when the caller does not want it
    // Jobs in size classes (ligands of at most 64 atoms, larger ones), each
    // with its own LDS limits, kernel variant and persistent launch; jobs
    // keep their indices through a per-group job map.
    std::vector<DockGroup> groups;
    std::vector<std::vector<int32_t>> group_jobs;   // per group: its plan jobs in job-map order
    std::vector<int32_t> job_group;   // per job: index into groups
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    pv_dock_out cached;
    bool have_graph;
};

namespace {

bool ctx_ok(const pv_ctx* c) { return c && c->magic == 0x70766378u; }

pv_status set_device(const pv_ctx* c)
{
    HIP_TRY(hipSetDevice(c->device), "hipSetDevice");
    return PV_OK;
}

GridDev grid_view(const pv_grids* g)
{
    GridDev v;
    v.maps = g->maps;
    v.dims = g->dims;
    v.geom = g->geom;
    v.map_off = g->map_off;
    v.n_boxes = g->n_boxes;
    v.kappa = g->kappa;
    return v;
}

LigDev lig_view(const pv_ligands* l)
{
    LigDev v;
    v.ligs = l->ligs;
    v.atoms = l->atoms;
    v.perm = l->perm;
    v.frags = l->frags;
    v.tors_frag = l->tors_frag;
    v.pairs = l->pairs;
    v.ell = l->ell;
    v.pslot = l->pslot;
    v.max_ell = l->max_ell;
    v.n_lig = l->n_lig;
    v.max_atoms = l->max_atoms;
    v.max_pairs = l->max_pairs;
    v.max_tors = l->max_tors;
    return v;
}

}  // namespace

extern "C" {

const char* pv_last_error(void) { return g_err.c_str(); }

int32_t pv_version(void) { return 102; }

pv_status pv_create(int32_t device, pv_ctx** out)
{
    if (!out) return fail(PV_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(PV_E_INVALID, "no such HIP device");
    HIP_TRY(hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    pv_ctx* c = new (std::nothrow) pv_ctx;
    if (!c) return fail(PV_E_NOMEM, "host allocation");
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    c->lds_per_block = (int)prop.sharedMemPerBlock;
    c->magic = 0x70766378u;
    // the allocation-free entry point's scratch: its address on this device,
    // taken once here with the device current (a failure is reported by
    // pv_dock_noalloc, the only call that needs it)
    c->scratch_err = noalloc_scratch(&c->scratch);
    *out = c;
    return PV_OK;
}

void pv_destroy(pv_ctx* c)
{
    if (!ctx_ok(c)) return;
    c->magic = 0;
    delete c;
}

// ------------------------------------------------------------------ grids
static pv_status lattice(const pv_box& B, int32_t dims[3], float origin[3], float ext[3])
{
    const double h = B.spacing;
    if (!(h > 0.0) || !std::isfinite(h)) return fail(PV_E_INVALID, "box spacing must be > 0");
    for (int a = 0; a < 3; ++a) {
        if (!(B.size[a] > 0.f) || !std::isfinite(B.size[a]) || !std::isfinite(B.center[a]))
            return fail(PV_E_INVALID, "box size must be > 0 and finite");
        const double n = std::ceil((double)B.size[a] / h) + 1.0;
        if (n > 2048.0) return fail(PV_E_RANGE, "more than 2048 lattice points on an axis");
        dims[a] = (int32_t)n;
        origin[a] = (float)((double)B.center[a] - 0.5 * (n - 1.0) * h);
        if (ext) ext[a] = (float)((n - 1.0) * h);
    }
    return PV_OK;
}

pv_status pv_box_lattice(const pv_box* box, int32_t dims[3], float origin[3])
{
    if (!box || !dims || !origin) return fail(PV_E_INVALID, "NULL argument");
    return lattice(*box, dims, origin, nullptr);
}

pv_status pv_build_grids(pv_ctx* ctx, int32_t n_rec, const float* rec_xyz, const uint8_t* rec_type,
                         const pv_box* boxes, int32_t n_boxes, float penalty_slope, void* stream,
                         pv_grids** out)
{
    if (!out) return fail(PV_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!ctx_ok(ctx)) return fail(PV_E_STATE, "invalid context");
    if (n_rec < 0) return fail(PV_E_INVALID, "n_rec < 0");
    if (n_rec > 0 && (!rec_xyz || !rec_type)) return fail(PV_E_INVALID, "receptor arrays are NULL");
    if (n_boxes < 1 || !boxes) return fail(PV_E_INVALID, "need at least one box");
    if (!(penalty_slope >= 0.f) || !std::isfinite(penalty_slope)) return fail(PV_E_INVALID, "penalty_slope must be finite and >= 0");
    for (int32_t r = 0; r < n_rec; ++r) {
        if (rec_type[r] >= kNTypes) return fail(PV_E_INVALID, "receptor atom type out of range");
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(rec_xyz[3 * r + a])) return fail(PV_E_INVALID, "non-finite receptor coordinate");
    }
    std::vector<int32_t> dims(4 * (size_t)n_boxes);
    std::vector<float> geom(8 * (size_t)n_boxes);
    std::vector<int64_t> off(n_boxes);
    std::vector<int32_t> tile_off(n_boxes + 1);
    int64_t total = 0, tiles = 0;
    for (int32_t b = 0; b < n_boxes; ++b) {
        const pv_box& B = boxes[b];
        int32_t d3[3];
        float o3[3], e3[3];
        pv_status ls = lattice(B, d3, o3, e3);
        if (ls != PV_OK) return ls;
        const double h = B.spacing;
        int64_t msz = 1;
        for (int a = 0; a < 3; ++a) {
            dims[4 * b + a] = d3[a];
            geom[8 * b + a] = o3[a];
            geom[8 * b + 5 + a] = e3[a];
            msz *= (int64_t)d3[a];
        }
        if (msz >= ((int64_t)1 << 24)) return fail(PV_E_RANGE, "a box's lattice has 2^24 points or more");
        dims[4 * b + 3] = 0;
        geom[8 * b + 3] = B.spacing;
        geom[8 * b + 4] = (float)(1.0 / h);
        off[b] = total;
        total += 8 * msz;
        tile_off[b] = (int32_t)tiles;
        tiles += (int64_t)((dims[4 * b] + kTileX - 1) / kTileX) * ((dims[4 * b + 1] + kTileY - 1) / kTileY) *
                 ((dims[4 * b + 2] + kTileZ - 1) / kTileZ);
        if (tiles > INT32_MAX) return fail(PV_E_RANGE, "too many lattice tiles");
    }
    tile_off[n_boxes] = (int32_t)tiles;
    // receptor atoms that can reach each box (8 A plus a margin)
    std::vector<float4> atoms;
    std::vector<int32_t> atom_off(n_boxes + 1, 0);
    for (int32_t b = 0; b < n_boxes; ++b) {
        atom_off[b] = (int32_t)atoms.size();
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = (double)geom[8 * b + a] - 8.05;
            hi[a] = (double)geom[8 * b + a] + (double)geom[8 * b + 5 + a] + 8.05;
        }
        for (int32_t r = 0; r < n_rec; ++r) {
            const float* x = rec_xyz + 3 * r;
            if (x[0] < lo[0] || x[0] > hi[0] || x[1] < lo[1] || x[1] > hi[1] || x[2] < lo[2] || x[2] > hi[2]) continue;
            float w;
            uint32_t t = rec_type[r];
            std::memcpy(&w, &t, 4);
            atoms.push_back(make_float4(x[0], x[1], x[2], w));
        }
    }
    atom_off[n_boxes] = (int32_t)atoms.size();
    pv_status st = set_device(ctx);
    if (st != PV_OK) return st;
    pv_grids* g = new (std::nothrow) pv_grids();
    if (!g) return fail(PV_E_NOMEM, "host allocation");
    g->ctx = ctx;
    g->n_boxes = n_boxes;
    g->kappa = penalty_slope;
    g->h_dims = dims;
    g->h_geom = geom;
    g->h_off = off;
    if ((st = upload(&g->maps, (const float*)nullptr, (size_t)total, "map allocation")) != PV_OK ||
        (st = upload(&g->dims, dims.data(), dims.size(), "grid tables")) != PV_OK ||
        (st = upload(&g->geom, geom.data(), geom.size(), "grid tables")) != PV_OK ||
        (st = upload(&g->map_off, off.data(), off.size(), "grid tables")) != PV_OK ||
        (st = upload(&g->atoms, atoms.data(), atoms.size(), "receptor upload")) != PV_OK ||
        (st = upload(&g->atom_off, atom_off.data(), atom_off.size(), "receptor upload")) != PV_OK ||
        (st = upload(&g->tile_off, tile_off.data(), tile_off.size(), "grid tables")) != PV_OK) {
        pv_grids_free(g);
        return st;
    }
    GridBuildArgs a;
    a.atoms = g->atoms;
    a.atom_off = g->atom_off;
    a.maps = g->maps;
    a.map_off = g->map_off;
    a.dims = g->dims;
    a.geom = g->geom;
    a.tile_off = g->tile_off;
    a.n_boxes = n_boxes;
    g->n_tiles = tiles;
    hipError_t e = launch_build_grids(a, tiles, (hipStream_t)stream);
    if (e != hipSuccess) {
        pv_grids_free(g);
        return hip_fail(e, "grid-map launch");
    }
    *out = g;
    return PV_OK;
}

pv_status pv_grids_rebuild(pv_grids* g, void* stream)
{
    if (!g) return fail(PV_E_INVALID, "grids is NULL");
    pv_status st = set_device(g->ctx);
    if (st != PV_OK) return st;
    GridBuildArgs a;
    a.atoms = g->atoms;
    a.atom_off = g->atom_off;
    a.maps = g->maps;
    a.map_off = g->map_off;
    a.dims = g->dims;
    a.geom = g->geom;
    a.tile_off = g->tile_off;
    a.n_boxes = g->n_boxes;
    HIP_TRY(launch_build_grids(a, g->n_tiles, (hipStream_t)stream), "grid-map launch");
    return PV_OK;
}

pv_status pv_grids_info(const pv_grids* g, int32_t box, int32_t dims[3], float origin[3], const float** dev_maps)
{
    if (!g) return fail(PV_E_INVALID, "grids is NULL");
    if (box < 0 || box >= g->n_boxes) return fail(PV_E_INVALID, "no such box");
    for (int a = 0; a < 3; ++a) {
        if (dims) dims[a] = g->h_dims[4 * box + a];
        if (origin) origin[a] = g->h_geom[8 * box + a];
    }
    if (dev_maps) *dev_maps = g->maps + g->h_off[box];
    return PV_OK;
}

pv_status pv_grids_copy(const pv_grids* g, int32_t box, float* dst, void* stream)
{
    if (!g || !dst) return fail(PV_E_INVALID, "NULL argument");
    if (box < 0 || box >= g->n_boxes) return fail(PV_E_INVALID, "no such box");
    pv_status st = set_device(g->ctx);
    if (st != PV_OK) return st;
    const size_t n = 8 * (size_t)g->h_dims[4 * box] * g->h_dims[4 * box + 1] * g->h_dims[4 * box + 2];
    HIP_TRY(hipMemcpyAsync(dst, g->maps + g->h_off[box], n * sizeof(float), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream),
            "hipMemcpyAsync");
    return PV_OK;
}

void pv_grids_free(pv_grids* g)
{
    if (!g) return;
    if (ctx_ok(g->ctx)) (void)hipSetDevice(g->ctx->device);
    dfree(g->maps); dfree(g->dims); dfree(g->geom); dfree(g->map_off);
    dfree(g->atoms); dfree(g->atom_off); dfree(g->tile_off);
    delete g;
}

// ------------------------------------------------------------------ ligands
pv_status pv_ligands_create(pv_ctx* ctx, int32_t n_lig, const int32_t* atom_off, const float* ref_xyz,
                            const uint8_t* type, const int32_t* bond_off, const int32_t* bonds,
                            const uint8_t* rotatable, pv_ligands** out)
{
    if (!out) return fail(PV_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!ctx_ok(ctx)) return fail(PV_E_STATE, "invalid context");
    if (n_lig < 1) return fail(PV_E_INVALID, "need at least one ligand");
    if (!atom_off || !ref_xyz || !type || !bond_off) return fail(PV_E_INVALID, "ligand arrays are NULL");
    if (atom_off[0] != 0 || bond_off[0] != 0) return fail(PV_E_INVALID, "offsets must start at 0");
    std::vector<DevLig> H(n_lig);
    std::vector<float> atoms;
    std::vector<int16_t> perm;
    std::vector<DevFrag> frags;
    std::vector<int8_t> tors_frag;
    std::vector<uint32_t> pairs;
    std::vector<uint32_t> ell;
    std::vector<uint32_t> pslot;
    auto* info = new (std::nothrow) std::vector<std::array<int32_t, 9>>(n_lig);
    if (!info) return fail(PV_E_NOMEM, "host allocation");
    int max_atoms = 0, max_pairs = 0, max_tors = 0, max_ell = 0;
    for (int32_t i = 0; i < n_lig; ++i) {
        const int32_t a0 = atom_off[i], a1 = atom_off[i + 1], b0 = bond_off[i], b1 = bond_off[i + 1];
        if (a1 < a0 || b1 < b0) { delete info; return fail(PV_E_INVALID, "offsets must not decrease"); }
        if (b1 > b0 && (!bonds || !rotatable)) { delete info; return fail(PV_E_INVALID, "bond arrays are NULL"); }
        LigModel M;
        std::string err;
        int rc = build_ligand_model(a1 - a0, ref_xyz + 3 * (size_t)a0, type + a0, b1 - b0,
                                    bonds ? bonds + 2 * (size_t)b0 : nullptr, rotatable ? rotatable + b0 : nullptr, M, err);
        if (rc != PV_OK) { delete info; return fail((pv_status)rc, "ligand " + std::to_string(i) + ": " + err); }
        DevLig& D = H[i];
        std::memset(&D, 0, sizeof(D));
        D.atom_base = (int32_t)perm.size();
        D.n_atoms = M.n;
        D.frag_base = (int32_t)frags.size();
        D.n_frag = M.nf;
        D.pair_base = (int32_t)pairs.size();
        D.n_pairs = M.np;
        D.tors_base = (int32_t)tors_frag.size();
        D.n_tors = M.nt;
        D.rounds = M.rounds;
        D.ell_base = (int32_t)ell.size();
        D.ell_w = M.ell_w;
        for (int a = 0; a < 3; ++a) D.anchor[a] = M.anchor[a];
        D.rot_amp_scale = (float)(1.0 / std::max((double)M.rg, 1e-3));
        atoms.insert(atoms.end(), M.ref.begin(), M.ref.end());
        for (int v : M.perm) perm.push_back((int16_t)v);
        frags.insert(frags.end(), M.frags.begin(), M.frags.end());
        for (int v : M.tors_frag) tors_frag.push_back((int8_t)v);
        pairs.insert(pairs.end(), M.pairs.begin(), M.pairs.end());
        ell.insert(ell.end(), M.ell.begin(), M.ell.end());
        pslot.insert(pslot.end(), M.pslot.begin(), M.pslot.end());
        max_ell = std::max(max_ell, M.ell_w * (M.n | 1));   // slot rows of an odd number of atoms
        (*info)[i] = {M.n, M.nf, M.nt, M.np, M.root_size, M.depth, 7 + M.nt, 0, M.ell_w * (M.n | 1)};
        max_atoms = std::max(max_atoms, M.n);
        max_pairs = std::max(max_pairs, M.np);
        max_tors = std::max(max_tors, M.nt);
    }
    // the device tables are addressed with 32-bit offsets
    for (size_t n : {perm.size(), frags.size(), tors_frag.size(), pairs.size(), ell.size(), pslot.size()})
        if (n > (size_t)INT32_MAX) { delete info; return fail(PV_E_RANGE, "ligand tables exceed 2^31 entries"); }
    pv_status st = set_device(ctx);
    if (st != PV_OK) { delete info; return st; }
    pv_ligands* L = new (std::nothrow) pv_ligands();
    if (!L) { delete info; return fail(PV_E_NOMEM, "host allocation"); }
    L->ctx = ctx;
    L->n_lig = n_lig;
    L->max_atoms = max_atoms;
    L->max_pairs = max_pairs;
    L->max_tors = max_tors;
    L->max_ell = max_ell;
    L->info = info;
    if ((st = upload(&L->ligs, H.data(), H.size(), "ligand upload")) != PV_OK ||
        (st = upload(&L->atoms, (const float4*)atoms.data(), atoms.size() / 4, "ligand upload")) != PV_OK ||
        (st = upload(&L->perm, perm.data(), perm.size(), "ligand upload")) != PV_OK ||
        (st = upload(&L->frags, frags.data(), frags.size(), "ligand upload")) != PV_OK ||
        (st = upload(&L->tors_frag, tors_frag.data(), tors_frag.size(), "ligand upload")) != PV_OK ||
        (st = upload(&L->pairs, pairs.data(), pairs.size(), "ligand upload")) != PV_OK ||
        (st = upload(&L->ell, ell.data(), ell.size(), "ligand upload")) != PV_OK ||
        (st = upload(&L->pslot, pslot.data(), pslot.size(), "ligand upload")) != PV_OK) {
        pv_ligands_free(L);
        return st;
    }
    *out = L;
    return PV_OK;
}

pv_status pv_ligands_info(const pv_ligands* l, int32_t lig, int32_t info[8])
{
    if (!l || !info) return fail(PV_E_INVALID, "NULL argument");
    if (lig < 0 || lig >= l->n_lig) return fail(PV_E_INVALID, "no such ligand");
    for (int k = 0; k < 8; ++k) info[k] = (*l->info)[lig][k];
    return PV_OK;
}

pv_status pv_ligand_describe(int32_t n_atoms, const float* ref_xyz, const uint8_t* type, int32_t n_bonds,
                             const int32_t* bonds, const uint8_t* rotatable, int32_t info[8], int32_t* pairs,
                             int32_t max_pairs, int32_t* frag)
{
    if (!info || !ref_xyz || !type || n_atoms < 0 || n_bonds < 0) return fail(PV_E_INVALID, "NULL or negative argument");
    if (n_bonds > 0 && (!bonds || !rotatable)) return fail(PV_E_INVALID, "bond arrays are NULL");
    LigModel M;
    std::string err;
    int rc = build_ligand_model(n_atoms, ref_xyz, type, n_bonds, bonds, rotatable, M, err);
    if (rc != PV_OK) return fail((pv_status)rc, err);
    const int32_t v[8] = {M.n, M.nf, M.nt, M.np, M.root_size, M.depth, 7 + M.nt, 0};
    for (int k = 0; k < 8; ++k) info[k] = v[k];
    if (pairs) {
        if (M.np > max_pairs) return fail(PV_E_RANGE, "more pairs than max_pairs");
        std::vector<std::pair<int, int>> pl;
        for (uint32_t pk : M.pairs) {
            int a = M.perm[pk & 0xff], b = M.perm[(pk >> 8) & 0xff];
            pl.push_back({std::min(a, b), std::max(a, b)});
        }
        std::sort(pl.begin(), pl.end());
        for (size_t i = 0; i < pl.size(); ++i) { pairs[2 * i] = pl[i].first; pairs[2 * i + 1] = pl[i].second; }
    }
    if (frag)
        for (int i = 0; i < M.n; ++i) {
            uint32_t w;
            std::memcpy(&w, &M.ref[4 * i + 3], 4);
            frag[M.perm[i]] = (int32_t)(w >> 8);
        }
    return PV_OK;
}

void pv_ligands_free(pv_ligands* l)
{
    if (!l) return;
    if (ctx_ok(l->ctx)) (void)hipSetDevice(l->ctx->device);
    dfree(l->ligs); dfree(l->atoms); dfree(l->perm); dfree(l->frags); dfree(l->tors_frag); dfree(l->pairs);
    dfree(l->ell); dfree(l->pslot);
    delete l->info;
    delete l;
}

// ------------------------------------------------------------------ score
static pv_status check_pair(pv_ctx* ctx, const pv_grids* g, const pv_ligands* l)
{
    if (!ctx_ok(ctx)) return fail(PV_E_STATE, "invalid context");
    if (!g || !l) return fail(PV_E_INVALID, "grids or ligands are NULL");
    if (g->ctx != ctx || l->ctx != ctx) return fail(PV_E_STATE, "handles belong to another context");
    return PV_OK;
}

pv_status pv_score_grad(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, int32_t n_poses,
                        const int32_t* lig_of_pose, const int32_t* box_of_pose, const float* dof,
                        int32_t dof_stride, const float* grad_energy, float* energy, float* e_parts,
                        float* grad_dof, float* xyz_out, float* grad_xyz, int32_t xyz_stride, void* stream)
{
    pv_status st = check_pair(ctx, grids, ligs);
    if (st != PV_OK) return st;
    if (n_poses < 0) return fail(PV_E_INVALID, "n_poses < 0");
    if (n_poses == 0) return PV_OK;
    if (!lig_of_pose || !box_of_pose || !dof) return fail(PV_E_INVALID, "input arrays are NULL");
    if (dof_stride < 7 + ligs->max_tors) return fail(PV_E_INVALID, "dof_stride < 7 + max torsions");
    if (dof_stride > 64) return fail(PV_E_RANGE, "dof_stride > 64");
    if ((xyz_out || grad_xyz) && xyz_stride < ligs->max_atoms) return fail(PV_E_INVALID, "xyz_stride < max atoms");
    if ((st = set_device(ctx)) != PV_OK) return st;
    ScoreArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = grid_view(grids);
    a.l = lig_view(ligs);
    a.n_poses = n_poses;
    a.lig_of_pose = lig_of_pose;
    a.box_of_pose = box_of_pose;
    a.dof = dof;
    a.dof_stride = dof_stride;
    a.from_xyz = 0;
    a.grad_energy = grad_energy;
    a.energy = energy;
    a.e_parts = e_parts;
    a.grad_dof = grad_dof;
    a.xyz_out = xyz_out;
    a.grad_xyz = grad_xyz;
    a.xyz_stride = xyz_stride;
    hipError_t e = launch_score(a, ctx->n_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "score launch");
    return PV_OK;
}

pv_status pv_score_grad_xyz(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, int32_t n_poses,
                            const int32_t* lig_of_pose, const int32_t* box_of_pose, const float* xyz,
                            int32_t xyz_stride, const float* grad_energy, float* energy, float* e_parts,
                            float* grad_xyz, void* stream)
{
    pv_status st = check_pair(ctx, grids, ligs);
    if (st != PV_OK) return st;
    if (n_poses < 0) return fail(PV_E_INVALID, "n_poses < 0");
    if (n_poses == 0) return PV_OK;
    if (!lig_of_pose || !box_of_pose || !xyz) return fail(PV_E_INVALID, "input arrays are NULL");
    if (xyz_stride < ligs->max_atoms) return fail(PV_E_INVALID, "xyz_stride < max atoms");
    if ((st = set_device(ctx)) != PV_OK) return st;
    ScoreArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = grid_view(grids);
    a.l = lig_view(ligs);
    a.n_poses = n_poses;
    a.lig_of_pose = lig_of_pose;
    a.box_of_pose = box_of_pose;
    a.dof = xyz;
    a.dof_stride = 0;
    a.from_xyz = 1;
    a.grad_energy = grad_energy;
    a.energy = energy;
    a.e_parts = e_parts;
    a.grad_xyz = grad_xyz;
    a.xyz_stride = xyz_stride;
    hipError_t e = launch_score(a, ctx->n_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "score launch");
    return PV_OK;
}

// ------------------------------------------------------------------ search
void pv_dock_params_default(pv_dock_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->chains = 8;
    p->steps = 100;
    p->bfgs_max_iter = 30;
    p->bfgs_m = 5;
    p->ls_max_trials = 10;
    p->refine_max_iter = 30;
    p->ls_rho = 1e-4f;
    p->ls_sigma = 0.1f;
    p->eps_grad = 1e-3f;
    p->eps_curv = 1e-6f;
    p->temperature = 1.2f;
    p->mut_pos_amp = 2.0f;
    p->mut_rot_amp = 2.0f;
    p->seed = 20043;
}

static pv_status check_search(const pv_dock_params* p, bool mc)
{
    if (!p) return fail(PV_E_INVALID, "params is NULL");
    if (mc && p->chains < 1) return fail(PV_E_INVALID, "chains < 1");
    if (mc && p->steps < 0) return fail(PV_E_INVALID, "steps < 0");
    if (p->bfgs_max_iter < 0 || (mc && p->refine_max_iter < 0)) return fail(PV_E_INVALID, "iteration caps must be >= 0");
    if (p->bfgs_m < 1 || p->bfgs_m > 8) return fail(PV_E_RANGE, "bfgs_m must be 1..8");
    if (p->ls_max_trials < 1 || p->ls_max_trials > 64) return fail(PV_E_RANGE, "ls_max_trials must be 1..64");
    if (!(p->ls_rho > 0.f && p->ls_rho < p->ls_sigma && p->ls_sigma < 1.f))
        return fail(PV_E_INVALID, "need 0 < ls_rho < ls_sigma < 1");
    if (!(p->eps_grad >= 0.f) || !(p->eps_curv >= 0.f)) return fail(PV_E_INVALID, "epsilons must be >= 0");
    if (mc && !(p->temperature > 0.f)) return fail(PV_E_INVALID, "temperature must be > 0");
    if (mc && (!(p->mut_pos_amp >= 0.f) || !(p->mut_rot_amp >= 0.f))) return fail(PV_E_INVALID, "amplitudes must be >= 0");
    if (p->consistency != 0 && p->consistency != 1) return fail(PV_E_INVALID, "consistency must be 0 or 1");
    if (p->max_evals < 0) return fail(PV_E_INVALID, "max_evals must be >= 0");
    return PV_OK;
}

static SearchParams to_sp(const pv_dock_params* p)
{
    SearchParams s;
    s.chains = p->chains;
    s.steps = p->steps;
    s.max_iter = p->bfgs_max_iter;
    s.m = p->bfgs_m;
    s.ls_max = p->ls_max_trials;
    s.refine_max_iter = p->refine_max_iter;
    s.rho = p->ls_rho;
    s.sigma = p->ls_sigma;
    s.eps_g = p->eps_grad;
    s.eps_c = p->eps_curv;
    s.temperature = p->temperature;
    s.pos_amp = p->mut_pos_amp;
    s.rot_amp = p->mut_rot_amp;
    s.flags = p->flags;
    s.consistency = p->consistency;
    s.seed = p->seed;
    s.max_evals = p->max_evals;
    return s;
}

pv_status pv_dock_plan(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, const pv_job* jobs,
                       int32_t n_jobs, const pv_dock_params* params, pv_plan** out)
{
    if (!out) return fail(PV_E_INVALID, "out is NULL");
    *out = nullptr;
    pv_status st = check_pair(ctx, grids, ligs);
    if (st != PV_OK) return st;
    if ((st = check_search(params, true)) != PV_OK) return st;
    static_assert(PV_DOCK_NO_INTRA_BOUND == kDockNoIntraBound, "the kernels' copy of the flag bit");
    if (params->flags & ~(PV_DOCK_TIMESTAMPS | PV_DOCK_GRAPH | PV_DOCK_LARGEST_FIRST | PV_DOCK_BOX_ORDER |
                          PV_DOCK_NO_INTRA_BOUND))
        return fail(PV_E_INVALID, "unknown dock flag");
    if (n_jobs < 0) return fail(PV_E_INVALID, "n_jobs < 0");
    if (n_jobs > 0 && !jobs) return fail(PV_E_INVALID, "jobs is NULL");
    if ((int64_t)n_jobs * params->chains > (int64_t)INT32_MAX) return fail(PV_E_RANGE, "jobs * chains too large");
    std::vector<int2> hj(n_jobs);
    for (int32_t j = 0; j < n_jobs; ++j) {
        if (jobs[j].ligand < 0 || jobs[j].ligand >= ligs->n_lig) return fail(PV_E_INVALID, "job names an unknown ligand");
        if (jobs[j].box < 0 || jobs[j].box >= grids->n_boxes) return fail(PV_E_INVALID, "job names an unknown box");
        hj[j] = make_int2(jobs[j].ligand, jobs[j].box);
    }
    if ((st = set_device(ctx)) != PV_OK) return st;
    pv_plan* P = new (std::nothrow) pv_plan();
    if (!P) return fail(PV_E_NOMEM, "host allocation");
    P->ctx = ctx;
    P->grids = grids;
    P->ligs = ligs;
    P->sp = to_sp(params);
    P->n_jobs = n_jobs;
    P->h_jobs = hj;
    const size_t nchain = (size_t)n_jobs * params->chains;
    if ((st = upload(&P->jobs, hj.data(), hj.size(), "job table")) != PV_OK ||
        (st = upload(&P->queue, (const uint32_t*)nullptr, 2, "queue")) != PV_OK ||
        (st = upload(&P->scratch_best, (const float*)nullptr, nchain, "scratch")) != PV_OK ||
        (st = upload(&P->scratch_evals, (const int64_t*)nullptr, nchain, "scratch")) != PV_OK ||
        (st = upload(&P->scratch_status, (const int32_t*)nullptr, nchain, "scratch")) != PV_OK) {
        pv_plan_free(P);
        return st;
    }
    // size classes: one atom per lane (at most 64 atoms) and two
    std::vector<int32_t> members[2];
    P->job_group.assign(n_jobs, 0);
    for (int32_t j = 0; j < n_jobs; ++j) members[(*ligs->info)[hj[j].x][0] > 64 ? 1 : 0].push_back(j);
    if (params->flags & PV_DOCK_LARGEST_FIRST) {
        // the queue hands out the jobs of a class in job-map order: the most
        // costly first (an evaluation's energy work: pairs tested, atoms,
        // torsions), so that the short ones fill the launch's tail
        auto cost = [&](int32_t j) {
            const auto& in = (*ligs->info)[hj[j].x];
            return 8 * (int64_t)in[3] + 48 * (int64_t)in[0] + 109 * (int64_t)in[2];
        };
        for (auto& m : members)
            std::stable_sort(m.begin(), m.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
    }
    if (params->flags & PV_DOCK_BOX_ORDER) {
        // one or two boxes' maps in flight at a time: each XCD's L2 holds
        // those rather than a slice of every box's
        for (auto& m : members)
            std::stable_sort(m.begin(), m.end(), [&](int32_t a, int32_t b) { return hj[a].y < hj[b].y; });
    }
    hipError_t e = hipSuccess;
    for (int g = 0; g < 2 && e == hipSuccess; ++g) {
        if (members[g].empty()) continue;
        DockGroup G;
        std::memset(&G, 0, sizeof(G));
        G.lv = lig_view(ligs);
        G.lv.max_atoms = G.lv.max_pairs = G.lv.max_tors = G.lv.max_ell = 0;
        for (int32_t j : members[g]) {
            const auto& in = (*ligs->info)[hj[j].x];
            G.lv.max_atoms = std::max(G.lv.max_atoms, in[0]);
            G.lv.max_tors = std::max(G.lv.max_tors, in[2]);
            G.lv.max_pairs = std::max(G.lv.max_pairs, in[3]);
            G.lv.max_ell = std::max(G.lv.max_ell, in[8]);
        }
        G.n_jobs = (int32_t)members[g].size();
        const int64_t items = (int64_t)G.n_jobs * params->chains;
        e = launch_shape(kKindDock, G.lv, items, ctx->n_cu, &G.shape);
        if (e == hipSuccess) e = launch_shape(kKindDock, G.lv, params->chains, ctx->n_cu, &G.plain_shape);
        if (e != hipSuccess) break;
        int64_t wg = params->workgroups > 0 ? params->workgroups : (int64_t)G.shape.per_cu * ctx->n_cu;
        G.workgroups = (int32_t)std::min<int64_t>(wg, std::max<int64_t>(items, 1));
        if ((st = upload(&G.job_map, members[g].data(), members[g].size(), "job map")) != PV_OK) {
            pv_plan_free(P);
            return st;
        }
        for (int32_t j : members[g]) P->job_group[j] = (int32_t)P->groups.size();
        P->groups.push_back(G);
        P->group_jobs.push_back(members[g]);
    }
    if (e != hipSuccess) { pv_plan_free(P); return hip_fail(e, "dock launch shape"); }
    e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { pv_plan_free(P); return hip_fail(e, "hipStreamCreate"); }
    *out = P;
    return PV_OK;
}

struct pv_sas {
    pv_ctx* ctx;
    int32_t n_rec;
    int32_t n_points;
    float4* atoms;   // (x, y, z, type bits)
    float4* pts;     // (x, y, z, atom index bits)
};

static DockArgs dock_args(pv_plan* P, const pv_dock_out* o, float* cbe, int64_t* cev, int32_t* cst)
{
    DockArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = grid_view(P->grids);
    a.l = lig_view(P->ligs);
    a.sp = P->sp;
    a.jobs = P->jobs;
    a.n_jobs = P->n_jobs;
    a.queue = P->queue;
    a.chain_best_e = cbe;
    a.chain_best_dof = o->chain_best_dof;
    a.chain_evals = cev;
    a.chain_pairs = o->chain_pairs;
    a.chain_grads = o->chain_grads;
    a.chain_bounded = o->chain_bounded;
    a.chain_status = cst;
    a.job_t_start = o->job_t_start;
    a.job_t_end = o->job_t_end;
    a.dof_stride = o->dof_stride;
    return a;
}

static pv_status check_out(const pv_plan* P, const pv_dock_out* o)
{
    if (!o) return fail(PV_E_INVALID, "out is NULL");
    if (o->chain_best_dof && (o->dof_stride < 7 + P->ligs->max_tors || o->dof_stride > 64))
        return fail(PV_E_INVALID, "dof_stride must be 7 + max torsions .. 64");
    if ((P->sp.flags & PV_DOCK_TIMESTAMPS) && (!o->job_t_start || !o->job_t_end))
        return fail(PV_E_INVALID, "timestamps requested without job_t_start / job_t_end");
    return PV_OK;
}

static hipError_t enqueue_batched(pv_plan* P, const pv_dock_out* o, hipStream_t s)
{
    float* cbe = o->chain_best_e ? o->chain_best_e : P->scratch_best;
    int64_t* cev = o->chain_evals ? o->chain_evals : P->scratch_evals;
    int32_t* cst = o->chain_status ? o->chain_status : P->scratch_status;
    hipError_t e = hipSuccess;
    if (P->sp.flags & PV_DOCK_TIMESTAMPS) {
        e = launch_reset_times(o->job_t_start, o->job_t_end, P->n_jobs, s);
        if (e != hipSuccess) return e;
    }
    for (size_t g = 0; g < P->groups.size(); ++g) {
        const DockGroup& G = P->groups[g];
        DockArgs a = dock_args(P, o, cbe, cev, cst);
        a.l = G.lv;
        a.job_map = G.job_map;
        a.queue = P->queue + g;
        a.job_begin = 0;
        a.n_items = (int64_t)G.n_jobs * P->sp.chains;
        a.persistent = 1;
        e = launch_reset_queue(a.queue, s);
        if (e == hipSuccess) e = launch_dock(a, G.shape, G.workgroups, s);
        if (e != hipSuccess) return e;
    }
    if (o->job_best_e || o->job_best_chain || o->job_evals || o->job_status)
        e = launch_job_reduce(cbe, cev, cst, P->n_jobs, P->sp.chains, o->job_best_e, o->job_best_chain, o->job_evals,
                              o->job_status, s);
    return e;
}

pv_status pv_dock_run(pv_plan* P, const pv_dock_out* o, void* stream)
{
    if (!P) return fail(PV_E_INVALID, "plan is NULL");
    pv_status st = check_out(P, o);
    if (st != PV_OK) return st;
    if ((st = set_device(P->ctx)) != PV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!(P->sp.flags & PV_DOCK_GRAPH)) {
        hipError_t e = enqueue_batched(P, o, s);
        if (e != hipSuccess) return hip_fail(e, "dock launch");
        return PV_OK;
    }
    if (!P->have_graph || std::memcmp(&P->cached, o, sizeof(*o)) != 0) {
        if (P->have_graph) {
            (void)hipGraphExecDestroy(P->exec);
            (void)hipGraphDestroy(P->graph);
            P->have_graph = false;
        }
        HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        hipError_t e = enqueue_batched(P, o, P->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(P->cap_stream, &g);
        if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(e, "dock launch (capture)"); }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e, "hipGraphInstantiate"); }
        P->graph = g;
        P->exec = x;
        P->cached = *o;
        P->have_graph = true;
    }
    HIP_TRY(hipGraphLaunch(P->exec, s), "hipGraphLaunch");
    return PV_OK;
}

pv_status pv_dock_run_plain(pv_plan* P, const pv_dock_out* o, void* stream)
{
    if (!P) return fail(PV_E_INVALID, "plan is NULL");
    pv_status st = check_out(P, o);
    if (st != PV_OK) return st;
    if ((st = set_device(P->ctx)) != PV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    float* cbe = o->chain_best_e ? o->chain_best_e : P->scratch_best;
    int64_t* cev = o->chain_evals ? o->chain_evals : P->scratch_evals;
    int32_t* cst = o->chain_status ? o->chain_status : P->scratch_status;
    if (P->sp.flags & PV_DOCK_TIMESTAMPS) HIP_TRY(launch_reset_times(o->job_t_start, o->job_t_end, P->n_jobs, s), "reset");
    for (int32_t j = 0; j < P->n_jobs; ++j) {
        const DockGroup& G = P->groups[P->job_group[j]];
        DockArgs a = dock_args(P, o, cbe, cev, cst);
        a.l = G.lv;
        a.job_begin = j;
        a.n_items = P->sp.chains;
        a.persistent = 0;
        HIP_TRY(launch_dock(a, G.plain_shape, 0, s), "dock launch");
    }
    if (o->job_best_e || o->job_best_chain || o->job_evals || o->job_status)
        HIP_TRY(launch_job_reduce(cbe, cev, cst, P->n_jobs, P->sp.chains, o->job_best_e, o->job_best_chain,
                                  o->job_evals, o->job_status, s),
                "job reduce");
    return PV_OK;
}

void pv_plan_free(pv_plan* P)
{
    if (!P) return;
    if (ctx_ok(P->ctx)) (void)hipSetDevice(P->ctx->device);
    if (P->have_graph) {
        (void)hipGraphExecDestroy(P->exec);
        (void)hipGraphDestroy(P->graph);
    }
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    dfree(P->jobs); dfree(P->queue); dfree(P->scratch_best); dfree(P->scratch_evals); dfree(P->scratch_status);
    for (DockGroup& G : P->groups) dfree(G.job_map);
    delete P;
}

// ------------------------------------------------------------------ schedules
static void drop_graph(pv_plan* P)
{
    if (P->have_graph) {
        (void)hipGraphExecDestroy(P->exec);
        (void)hipGraphDestroy(P->graph);
        P->have_graph = false;
    }
}

pv_status pv_plan_groups(const pv_plan* P, int32_t* n_groups)
{
    if (!P || !n_groups) return fail(PV_E_INVALID, "plan or output is NULL");
    *n_groups = (int32_t)P->groups.size();
    return PV_OK;
}

pv_status pv_plan_schedule(const pv_plan* P, int32_t group, pv_schedule* out)
{
    if (!P || !out) return fail(PV_E_INVALID, "plan or output is NULL");
    if (group < 0 || group >= (int32_t)P->groups.size()) return fail(PV_E_RANGE, "no such size class");
    const DockGroup& G = P->groups[group];
    out->variant = G.shape.variant;
    out->workgroups = G.workgroups;
    out->lds_bytes = G.shape.lds;
    out->per_cu = G.shape.per_cu;
    out->n_jobs = G.n_jobs;
    return PV_OK;
}

// Shape and width of `variant` for a size class; workgroups 0 = all the CUs
// hold, capped by the class's work.  The device must be current.
static pv_status group_shape(const pv_plan* P, int32_t group, int32_t variant, int32_t workgroups, LaunchShape* sh,
                             int32_t* wg)
{
    const DockGroup& G = P->groups[group];
    const hipError_t e = launch_shape_variant(kKindDock, G.lv, variant, sh);
    if (e == hipErrorInvalidValue) return fail(PV_E_INVALID, "variant not available for this size class");
    if (e != hipSuccess || sh->lds > P->ctx->lds_per_block)
        return fail(PV_E_RANGE, "a workgroup of this variant does not fit a CU");
    const int64_t items = (int64_t)G.n_jobs * P->sp.chains;
    if (workgroups < 0 || workgroups > items) return fail(PV_E_RANGE, "workgroups must be 0 .. jobs x chains of the class");
    *wg = workgroups > 0 ? workgroups
                         : (int32_t)std::min<int64_t>((int64_t)sh->per_cu * P->ctx->n_cu, std::max<int64_t>(items, 1));
    return PV_OK;
}

pv_status pv_plan_set_schedule(pv_plan* P, int32_t group, int32_t variant, int32_t workgroups)
{
    if (!P) return fail(PV_E_INVALID, "plan is NULL");
    if (group < 0 || group >= (int32_t)P->groups.size()) return fail(PV_E_RANGE, "no such size class");
    pv_status st = set_device(P->ctx);
    if (st != PV_OK) return st;
    LaunchShape sh;
    int32_t wg = 0;
    if ((st = group_shape(P, group, variant, workgroups, &sh, &wg)) != PV_OK) return st;
    P->groups[group].shape = sh;
    P->groups[group].workgroups = wg;
    drop_graph(P);
    return PV_OK;
}

static bool same_key(const TuneEntry& a, const TuneEntry& b)
{
    return a.max_atoms == b.max_atoms && a.max_pairs == b.max_pairs && a.max_ell == b.max_ell &&
           a.max_tors == b.max_tors && a.items == b.items && a.steps == b.steps && a.max_iter == b.max_iter &&
           a.refine_max_iter == b.refine_max_iter && a.m == b.m && a.ls_max == b.ls_max &&
           a.consistency == b.consistency;
}

pv_status pv_dock_autotune(pv_plan* P, int32_t tune_steps, int32_t repeats, void* stream, pv_tune_result* results,
                           int32_t max_results, int32_t* n_results)
{
    if (n_results) *n_results = 0;
    if (!P) return fail(PV_E_INVALID, "plan is NULL");
    if (tune_steps < 1) return fail(PV_E_INVALID, "tune_steps < 1");
    if (repeats < 1 || repeats > 100) return fail(PV_E_RANGE, "repeats must be 1 .. 100");
    if (max_results < 0 || (max_results > 0 && !results)) return fail(PV_E_INVALID, "results is NULL");
    pv_status st = set_device(P->ctx);
    if (st != PV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    int32_t written = 0;
    auto put = [&](const pv_tune_result& r) -> int32_t {
        if (written >= max_results) return -1;
        results[written] = r;
        return written++;
    };
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    auto done = [&](pv_status r) {
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
        drop_graph(P);
        if (n_results) *n_results = written;
        return r;
    };
    if (e != hipSuccess) return done(hip_fail(e, "hipEventCreate"));
    const int32_t chains = P->sp.chains;
    std::vector<int64_t> hev((size_t)P->n_jobs * chains);
    pv_dock_out none;
    std::memset(&none, 0, sizeof(none));
    for (size_t g = 0; g < P->groups.size(); ++g) {
        DockGroup& G = P->groups[g];
        const int64_t items = (int64_t)G.n_jobs * chains;
        TuneEntry key = {G.lv.max_atoms, G.lv.max_pairs, G.lv.max_ell, G.lv.max_tors, items, tune_steps,
                         P->sp.max_iter, P->sp.refine_max_iter, P->sp.m, P->sp.ls_max, P->sp.consistency, 0, 0};
        bool cached = false;
        {
            std::lock_guard<std::mutex> lock(P->ctx->tune_mu);
            for (const TuneEntry& t : P->ctx->tune)
                if (same_key(t, key)) { key.variant = t.variant; key.workgroups = t.workgroups; cached = true; break; }
        }
        if (cached) {
            LaunchShape sh;
            int32_t wg = 0;
            if ((st = group_shape(P, (int32_t)g, key.variant, key.workgroups, &sh, &wg)) != PV_OK) return done(st);
            G.shape = sh;
            G.workgroups = wg;
            put(pv_tune_result{(int32_t)g, sh.variant, wg, 1, 1, 0.f, 0.0});
            continue;
        }
        // candidates: the current schedule first, then every legal variant
        // at 1, 3/4 and 1/2 of the width the CUs hold
        std::vector<std::pair<LaunchShape, int32_t>> cand;
        cand.push_back({G.shape, G.workgroups});
        for (int v = G.lv.max_atoms <= 64 ? 0 : 2; v <= 2; ++v) {
            LaunchShape sh;
            if (launch_shape_variant(kKindDock, G.lv, v, &sh) != hipSuccess || sh.lds > P->ctx->lds_per_block) continue;
            const int64_t full = std::min<int64_t>((int64_t)sh.per_cu * P->ctx->n_cu, std::max<int64_t>(items, 1));
            for (int q = 4; q >= 2; --q) {
                const int32_t wg = (int32_t)std::max<int64_t>(1, (full * q + 3) / 4);
                bool seen = false;
                for (const auto& c : cand) seen = seen || (c.first.variant == v && c.second == wg);
                if (!seen) cand.push_back({sh, wg});
            }
        }
        // every candidate runs on the class's first jobs in job-map order:
        // enough chains to fill the widest candidate kTuneFill times (all of
        // the class when it is smaller), so the tuning cost does not grow
        // with the batch
        int64_t widest = 1;
        for (const auto& c : cand) widest = std::max<int64_t>(widest, c.second);
        const int64_t t_items = std::min<int64_t>(items, (kTuneFill * widest + chains - 1) / chains * chains);
        const int32_t t_jobs = (int32_t)(t_items / chains);
        size_t best = 0;
        double best_rate = -1.0;
        std::vector<int32_t> slot(cand.size(), -1);
        for (size_t k = 0; k < cand.size(); ++k) {
            DockArgs a = dock_args(P, &none, P->scratch_best, P->scratch_evals, P->scratch_status);
            a.sp.steps = tune_steps;
            a.sp.flags &= ~PV_DOCK_TIMESTAMPS;
            a.l = G.lv;
            a.job_map = G.job_map;
            a.queue = P->queue + g;
            a.job_begin = 0;
            a.n_items = t_items;
            a.persistent = 1;
            float best_ms = 0.f;
            for (int r = 0; r < repeats; ++r) {
                e = launch_reset_queue(a.queue, s);
                if (e == hipSuccess) e = hipEventRecord(t0, s);
                if (e == hipSuccess) e = launch_dock(a, cand[k].first, cand[k].second, s);
                if (e == hipSuccess) e = hipEventRecord(t1, s);
                if (e == hipSuccess) e = hipEventSynchronize(t1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                if (e != hipSuccess) return done(hip_fail(e, "autotune launch"));
                best_ms = r == 0 ? ms : std::min(best_ms, ms);
            }
            e = hipMemcpy(hev.data(), P->scratch_evals, hev.size() * sizeof(int64_t), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return done(hip_fail(e, "autotune evaluation counts"));
            int64_t ev = 0;
            for (int32_t q = 0; q < t_jobs; ++q) {
                const int32_t j = P->group_jobs[g][q];
                for (int32_t c = 0; c < chains; ++c) ev += hev[(size_t)j * chains + c];
            }
            const double rate = best_ms > 0.f ? (double)ev / (best_ms * 1e-3) : 0.0;
            slot[k] = put(pv_tune_result{(int32_t)g, cand[k].first.variant, cand[k].second, 0, 0, best_ms, rate});
            if (rate > best_rate) { best_rate = rate; best = k; }
        }
        G.shape = cand[best].first;
        G.workgroups = cand[best].second;
        if (slot[best] >= 0) results[slot[best]].chosen = 1;
        key.variant = G.shape.variant;
        key.workgroups = G.workgroups;
        std::lock_guard<std::mutex> lock(P->ctx->tune_mu);
        if (P->ctx->tune.size() >= kTuneMemory) P->ctx->tune.erase(P->ctx->tune.begin());   // the oldest goes
        P->ctx->tune.push_back(key);
    }
    return done(PV_OK);
}

pv_status pv_fma_peak(pv_ctx* ctx, int32_t iters, float* dev_out, int32_t n_out, void* stream)
{
    if (!ctx_ok(ctx)) return fail(PV_E_STATE, "invalid context");
    if (!dev_out) return fail(PV_E_INVALID, "dev_out is NULL");
    if (iters < 1 || n_out < 256 || n_out % 256 != 0)
        return fail(PV_E_INVALID, "need iters >= 1 and n_out a positive multiple of 256");
    pv_status st = set_device(ctx);
    if (st != PV_OK) return st;
    HIP_TRY(launch_fma_peak(dev_out, n_out, iters, (hipStream_t)stream), "fma peak launch");
    return PV_OK;
}

pv_status pv_dock(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, const pv_job* jobs, int32_t n_jobs,
                  const pv_dock_params* params, const pv_dock_out* out, void* stream)
{
    pv_plan* P = nullptr;
    pv_status st = pv_dock_plan(ctx, grids, ligs, jobs, n_jobs, params, &P);
    if (st != PV_OK) return st;
    st = pv_dock_run(P, out, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    pv_plan_free(P);
    if (st != PV_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return PV_OK;
}

// ------------------------------------------------------------------ allocation-free dock
// pv_dock without any allocation: the job table, the per-class job maps, the
// queue counters and (when the caller takes none) the per-chain best
// energies and evaluation counts live in the device's scratch array.  The
// size classes, their LDS limits, variants and widths are those pv_dock_plan
// gives the same jobs, so the outputs equal pv_dock's bit for bit.
static std::mutex g_noalloc_mu[64];   // one per device: calls on a device share its scratch

pv_status pv_dock_noalloc(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, const pv_job* jobs,
                          int32_t n_jobs, const pv_dock_params* params, const pv_dock_out* out, void* stream)
{
    pv_status st = check_pair(ctx, grids, ligs);
    if (st != PV_OK) return st;
    if ((st = check_search(params, true)) != PV_OK) return st;
    if (params->flags & ~PV_DOCK_TIMESTAMPS) return fail(PV_E_INVALID, "only PV_DOCK_TIMESTAMPS is accepted here");
    if (!out) return fail(PV_E_INVALID, "out is NULL");
    if (n_jobs < 0) return fail(PV_E_INVALID, "n_jobs < 0");
    if (n_jobs > 0 && !jobs) return fail(PV_E_INVALID, "jobs is NULL");
    if (n_jobs > kNoAllocMaxJobs) return fail(PV_E_RANGE, "n_jobs above PV_NOALLOC_MAX_JOBS");
    if ((int64_t)n_jobs * params->chains > kNoAllocMaxChains)
        return fail(PV_E_RANGE, "n_jobs * chains above PV_NOALLOC_MAX_CHAINS");
    if (out->chain_best_dof && (out->dof_stride < 7 + ligs->max_tors || out->dof_stride > 64))
        return fail(PV_E_INVALID, "dof_stride must be 7 + max torsions .. 64");
    if ((params->flags & PV_DOCK_TIMESTAMPS) && (!out->job_t_start || !out->job_t_end))
        return fail(PV_E_INVALID, "timestamps requested without job_t_start / job_t_end");
    // size classes on the host, as pv_dock_plan forms them: counts and the
    // LDS limits of each (no allocation)
    int32_t cnt[2] = {0, 0};
    LigDev lv[2] = {lig_view(ligs), lig_view(ligs)};
    for (int g = 0; g < 2; ++g) lv[g].max_atoms = lv[g].max_pairs = lv[g].max_tors = lv[g].max_ell = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
        if (jobs[j].ligand < 0 || jobs[j].ligand >= ligs->n_lig) return fail(PV_E_INVALID, "job names an unknown ligand");
        if (jobs[j].box < 0 || jobs[j].box >= grids->n_boxes) return fail(PV_E_INVALID, "job names an unknown box");
        const auto& in = (*ligs->info)[jobs[j].ligand];
        LigDev& v = lv[in[0] > 64 ? 1 : 0];
        ++cnt[in[0] > 64 ? 1 : 0];
        v.max_atoms = std::max(v.max_atoms, in[0]);
        v.max_tors = std::max(v.max_tors, in[2]);
        v.max_pairs = std::max(v.max_pairs, in[3]);
        v.max_ell = std::max(v.max_ell, in[8]);
    }
    if ((st = set_device(ctx)) != PV_OK) return st;
    if (!ctx->scratch) return hip_fail(ctx->scratch_err, "scratch address (hipGetSymbolAddress)");
    if (ctx->device < 0 || ctx->device >= 64) return fail(PV_E_RANGE, "device index above 63");
    LaunchShape sh[2];
    int32_t width[2] = {0, 0};
    for (int g = 0; g < 2; ++g) {
        if (!cnt[g]) continue;
        const int64_t items = (int64_t)cnt[g] * params->chains;
        hipError_t e = launch_shape(kKindDock, lv[g], items, ctx->n_cu, &sh[g]);
        if (e != hipSuccess) return hip_fail(e, "dock launch shape");
        const int64_t wg = params->workgroups > 0 ? params->workgroups : (int64_t)sh[g].per_cu * ctx->n_cu;
        width[g] = (int32_t)std::min<int64_t>(wg, std::max<int64_t>(items, 1));
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu[ctx->device]);
    const NoAllocLayout W = noalloc_layout(ctx->scratch);
    hipStream_t s = (hipStream_t)stream;
    float* cbe = out->chain_best_e ? out->chain_best_e : W.best;
    int64_t* cev = out->chain_evals ? out->chain_evals : W.evals;
    int32_t* cst = out->chain_status ? out->chain_status : W.status;
    if (n_jobs > 0) {
        static_assert(sizeof(pv_job) == sizeof(int2), "pv_job is two int32");
        HIP_TRY(hipMemcpyAsync(W.jobs, jobs, (size_t)n_jobs * sizeof(int2), hipMemcpyHostToDevice, s), "job table copy");
        HIP_TRY(launch_class_map(W.jobs, n_jobs, ligs->ligs, cnt[0], W.map, W.queues, s), "class map");
    }
    if (params->flags & PV_DOCK_TIMESTAMPS)
        HIP_TRY(launch_reset_times(out->job_t_start, out->job_t_end, n_jobs, s), "reset");
    for (int g = 0; g < 2; ++g) {
        if (!cnt[g]) continue;
        DockArgs a;
        std::memset(&a, 0, sizeof(a));
        a.g = grid_view(grids);
        a.l = lv[g];
        a.sp = to_sp(params);
        a.jobs = W.jobs;
        a.n_jobs = n_jobs;
        a.queue = W.queues + g;
        a.job_map = W.map + (g ? cnt[0] : 0);
        a.n_items = (int64_t)cnt[g] * params->chains;
        a.persistent = 1;
        a.chain_best_e = cbe;
        a.chain_best_dof = out->chain_best_dof;
        a.chain_evals = cev;
        a.chain_pairs = out->chain_pairs;
        a.chain_grads = out->chain_grads;
        a.chain_bounded = out->chain_bounded;
        a.chain_status = cst;
        a.job_t_start = out->job_t_start;
        a.job_t_end = out->job_t_end;
        a.dof_stride = out->dof_stride;
        HIP_TRY(launch_dock(a, sh[g], width[g], s), "dock launch");
    }
    if (out->job_best_e || out->job_best_chain || out->job_evals || out->job_status)
        HIP_TRY(launch_job_reduce(cbe, cev, cst, n_jobs, params->chains, out->job_best_e, out->job_best_chain,
                                  out->job_evals, out->job_status, s),
                "job reduce");
    // the scratch is reused by the next call on this device: return only
    // once this call's work (and the read of the caller's host jobs) is done
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    return PV_OK;
}

pv_status pv_local_opt(pv_ctx* ctx, const pv_grids* grids, const pv_ligands* ligs, int32_t n_poses,
                       const int32_t* lig_of_pose, const int32_t* box_of_pose, const float* dof_in,
                       int32_t dof_stride, const pv_dock_params* params, float* dof_out, float* energy,
                       int64_t* n_evals, void* stream)
{
    pv_status st = check_pair(ctx, grids, ligs);
    if (st != PV_OK) return st;
    if ((st = check_search(params, false)) != PV_OK) return st;
    if (n_poses < 0) return fail(PV_E_INVALID, "n_poses < 0");
    if (n_poses == 0) return PV_OK;
    if (!lig_of_pose || !box_of_pose || !dof_in || !dof_out) return fail(PV_E_INVALID, "pose arrays are NULL");
    if (dof_stride < 7 + ligs->max_tors || dof_stride > 64) return fail(PV_E_INVALID, "dof_stride must be 7 + max torsions .. 64");
    if ((st = set_device(ctx)) != PV_OK) return st;
    OptArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = grid_view(grids);
    a.l = lig_view(ligs);
    a.sp = to_sp(params);
    a.n_poses = n_poses;
    a.lig_of_pose = lig_of_pose;
    a.box_of_pose = box_of_pose;
    a.dof_in = dof_in;
    a.dof_stride = dof_stride;
    a.dof_out = dof_out;
    a.energy = energy;
    a.n_evals = n_evals;
    hipError_t e = launch_local_opt(a, ctx->n_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "local-opt launch");
    return PV_OK;
}

void pv_output_params_default(pv_output_params* p)
{
    if (!p) return;
    p->modes = 20;
    p->refine_max_iter = 30;
    p->rmsd_cut = 1.0f;
    p->affinity_w = 0.0585f;
}

pv_status pv_output_stage(pv_plan* P, const float* chain_best_e, const float* chain_best_dof, int32_t in_stride,
                          const pv_output_params* params, const pv_modes_out* out, void* stream)
{
    if (!P) return fail(PV_E_INVALID, "plan is NULL");
    if (!params || !out) return fail(PV_E_INVALID, "params or out is NULL");
    if (!chain_best_e || !chain_best_dof) return fail(PV_E_INVALID, "chain bests are NULL");
    if (!out->n_modes || !out->mode_chain || !out->mode_e) return fail(PV_E_INVALID, "n_modes, mode_chain, mode_e are required");
    if (params->modes < 1 || params->modes > PV_MAX_MODES) return fail(PV_E_RANGE, "modes must be 1..32");
    if (params->refine_max_iter < 0) return fail(PV_E_INVALID, "refine_max_iter < 0");
    if (!(params->rmsd_cut >= 0.f) || !std::isfinite(params->rmsd_cut)) return fail(PV_E_INVALID, "rmsd_cut must be finite and >= 0");
    if (!std::isfinite(params->affinity_w) || !(params->affinity_w >= 0.f)) return fail(PV_E_INVALID, "affinity_w must be finite and >= 0");
    const int need = 7 + P->ligs->max_tors;
    if (in_stride < need || in_stride > 64) return fail(PV_E_INVALID, "in_stride must be 7 + max torsions .. 64");
    if (out->mode_dof && (out->dof_stride < need || out->dof_stride > 64))
        return fail(PV_E_INVALID, "dof_stride must be 7 + max torsions .. 64");
    if (P->sp.chains > PV_MAX_OUTPUT_CHAINS) return fail(PV_E_RANGE, "the output stage takes at most 4096 chains per job");
    pv_status st = set_device(P->ctx);
    if (st != PV_OK) return st;
    OutputArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = grid_view(P->grids);
    a.l = lig_view(P->ligs);
    a.sp = P->sp;
    a.jobs = P->jobs;
    a.n_jobs = P->n_jobs;
    a.chains = P->sp.chains;
    a.chain_e = chain_best_e;
    a.chain_dof = chain_best_dof;
    a.in_stride = in_stride;
    a.modes = params->modes;
    a.refine_max_iter = params->refine_max_iter;
    a.rmsd_cut = params->rmsd_cut;
    a.affinity_w = params->affinity_w;
    a.n_modes = out->n_modes;
    a.mode_chain = out->mode_chain;
    a.mode_e = out->mode_e;
    a.mode_affinity = out->mode_affinity;
    a.mode_dof = out->mode_dof;
    a.out_stride = out->dof_stride;
    if (output_lds_bytes(a.l, a.chains, a.modes) > P->ctx->lds_per_block)
        return fail(PV_E_RANGE, "chains, modes and ligand size need more LDS than one workgroup has");
    hipError_t e = launch_output(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "output-stage launch");
    return PV_OK;
}

pv_status pv_sas_build(pv_ctx* ctx, int32_t n_rec, const float* rec_xyz, const uint8_t* rec_type, int32_t n_dirs,
                       const float* dirs, float probe, void* stream, pv_sas** out)
{
    if (!out) return fail(PV_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!ctx_ok(ctx)) return fail(PV_E_INVALID, "bad context");
    if (n_rec < 0) return fail(PV_E_INVALID, "n_rec < 0");
    if (n_rec > 0 && (!rec_xyz || !rec_type)) return fail(PV_E_INVALID, "receptor arrays are NULL");
    if (n_dirs < 1 || n_dirs > PV_MAX_SAS_DIRS) return fail(PV_E_RANGE, "n_dirs must be 1..4096");
    if (!dirs) return fail(PV_E_INVALID, "dirs is NULL");
    if (!(probe >= 0.f) || !std::isfinite(probe)) return fail(PV_E_INVALID, "probe must be finite and >= 0");
    const int64_t n_cand = (int64_t)n_rec * n_dirs;
    if (n_cand > (int64_t)INT32_MAX) return fail(PV_E_RANGE, "atoms x directions too large");
    std::vector<float4> ha((size_t)std::max(n_rec, 1));
    for (int32_t a = 0; a < n_rec; ++a) {
        if (rec_type[a] >= kNTypes) return fail(PV_E_INVALID, "receptor type out of range");
        const float x = rec_xyz[3 * a], y = rec_xyz[3 * a + 1], z = rec_xyz[3 * a + 2];
        if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return fail(PV_E_INVALID, "non-finite coordinate");
        uint32_t tb = rec_type[a];
        float w;
        std::memcpy(&w, &tb, 4);
        ha[a] = make_float4(x, y, z, w);
    }
    for (int32_t k = 0; k < 3 * n_dirs; ++k)
        if (!std::isfinite(dirs[k])) return fail(PV_E_INVALID, "non-finite direction");
    pv_status st = set_device(ctx);
    if (st != PV_OK) return st;
    pv_sas* h = new (std::nothrow) pv_sas();
    if (!h) return fail(PV_E_NOMEM, "host allocation");
    h->ctx = ctx;
    h->n_rec = n_rec;
    hipStream_t s = (hipStream_t)stream;
    const int bs = sas_block_size();
    const int64_t n_blocks = (n_cand + bs - 1) / bs;
    float* ddirs = nullptr;
    float4* cand = nullptr;
    uint8_t* keep = nullptr;
    int32_t* bcount = nullptr;
    int32_t* boff = nullptr;
    auto cleanup = [&]() { dfree(ddirs); dfree(cand); dfree(keep); dfree(bcount); dfree(boff); };
    if ((st = upload(&h->atoms, ha.data(), ha.size(), "receptor")) != PV_OK ||
        (st = upload(&ddirs, dirs, (size_t)3 * n_dirs, "directions")) != PV_OK ||
        (st = upload(&cand, (const float4*)nullptr, (size_t)std::max<int64_t>(n_cand, 1), "candidates")) != PV_OK ||
        (st = upload(&keep, (const uint8_t*)nullptr, (size_t)std::max<int64_t>(n_cand, 1), "candidates")) != PV_OK ||
        (st = upload(&bcount, (const int32_t*)nullptr, (size_t)std::max<int64_t>(n_blocks, 1), "counts")) != PV_OK) {
        cleanup();
        pv_sas_free(h);
        return st;
    }
    hipError_t e = launch_sas_candidates(h->atoms, n_rec, ddirs, n_dirs, probe, n_cand, cand, keep, bcount, s);
    std::vector<int32_t> hc((size_t)std::max<int64_t>(n_blocks, 1), 0);
    if (e == hipSuccess && n_blocks > 0)
        e = hipMemcpyAsync(hc.data(), bcount, sizeof(int32_t) * n_blocks, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { cleanup(); pv_sas_free(h); return hip_fail(e, "surface candidates"); }
    int64_t total = 0;
    for (int64_t b = 0; b < n_blocks; ++b) {
        const int32_t c = hc[b];
        hc[b] = (int32_t)total;
        total += c;
    }
    h->n_points = (int32_t)total;
    if ((st = upload(&boff, hc.data(), hc.size(), "offsets")) != PV_OK ||
        (st = upload(&h->pts, (const float4*)nullptr, (size_t)std::max<int64_t>(total, 1), "points")) != PV_OK) {
        cleanup();
        pv_sas_free(h);
        return st;
    }
    e = launch_sas_scatter(cand, keep, boff, n_cand, h->pts, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) { pv_sas_free(h); return hip_fail(e, "surface points"); }
    *out = h;
    return PV_OK;
}

pv_status pv_sas_info(const pv_sas* h, int32_t* n_points)
{
    if (!h || !n_points) return fail(PV_E_INVALID, "handle or output is NULL");
    *n_points = h->n_points;
    return PV_OK;
}

pv_status pv_sas_copy(const pv_sas* h, float* xyz, int32_t* atom, void* stream)
{
    if (!h) return fail(PV_E_INVALID, "handle is NULL");
    if (h->n_points == 0) return PV_OK;
    pv_status st = set_device(h->ctx);
    if (st != PV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (xyz)
        HIP_TRY(hipMemcpy2DAsync(xyz, 12, h->pts, 16, 12, h->n_points, hipMemcpyDeviceToDevice, s), "copy points");
    if (atom)
        HIP_TRY(hipMemcpy2DAsync(atom, 4, (const char*)h->pts + 12, 16, 4, h->n_points, hipMemcpyDeviceToDevice, s),
                "copy atoms");
    return PV_OK;
}

pv_status pv_sas_features(const pv_sas* h, float* features, void* stream)
{
    if (!h) return fail(PV_E_INVALID, "handle is NULL");
    if (h->n_points == 0) return PV_OK;
    if (!features) return fail(PV_E_INVALID, "features is NULL");
    pv_status st = set_device(h->ctx);
    if (st != PV_OK) return st;
    HIP_TRY(launch_sas_features(h->atoms, h->n_rec, h->pts, h->n_points, features, (hipStream_t)stream),
            "surface features");
    return PV_OK;
}

void pv_sas_free(pv_sas* h)
{
    if (!h) return;
    if (h->ctx) (void)hipSetDevice(h->ctx->device);
    dfree(h->atoms);
    dfree(h->pts);
    delete h;
}

pv_status pv_launch_info(pv_ctx* ctx, const pv_ligands* ligs, int32_t kind, int64_t items, int32_t* variant,
                         int32_t* lds_bytes, int32_t* per_cu)
{
    if (!ctx_ok(ctx)) return fail(PV_E_INVALID, "bad context");
    if (!ligs) return fail(PV_E_INVALID, "ligands are NULL");
    static_assert(PV_KIND_DOCK == kKindDock && PV_KIND_SCORE == kKindScore && PV_KIND_LOCAL_OPT == kKindOpt,
                  "kernel kinds");
    if (kind < PV_KIND_DOCK || kind > PV_KIND_LOCAL_OPT) return fail(PV_E_INVALID, "unknown kernel kind");
    if (items < 0) return fail(PV_E_INVALID, "items < 0");
    pv_status st = set_device(ctx);
    if (st != PV_OK) return st;
    LaunchShape sh;
    hipError_t e = launch_shape(kind, lig_view(ligs), items, ctx->n_cu, &sh);
    if (e != hipSuccess) return hip_fail(e, "launch shape");
    if (variant) *variant = sh.variant;
    if (lds_bytes) *lds_bytes = sh.lds;
    if (per_cu) *per_cu = sh.per_cu;
    return PV_OK;
}

}  // extern "C"
