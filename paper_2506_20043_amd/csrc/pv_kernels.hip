// pv_kernels.hip -- gfx950 kernels of the docking hot path.
//
//  * grid maps ("Kernel 1" of the paper: one map per ligand atom type over
//    each pocket box, Methods "Accelerated Docking" and Supplementary
//    Algorithm 2, first step): FP32 VALU, lattice tiles of 16x4x4 points per
//    workgroup, receptor atoms culled per tile into LDS;
//  * pose evaluation (Eq. qvina_eq_1 forward kinematics, Eq. qvina_eq_3
//    score): one wave64 per pose, lanes over fragments for the frame tree,
//    over atoms for the trilinear gathers and over intra pairs, LDS force
//    accumulation and a wave scan that carries force and torque back to the
//    torsions;
//  * RILC-BFGS (Eqs. qvina_eq_6 .. qvina_eq_12) with the tangent-space
//    vectors spread one component per lane;
//  * Monte Carlo chains (Supplementary Algorithm 2, Eq. qvina_eq_13) in a
//    persistent launch whose waves pull (job, chain) items from a device
//    queue, with Philox4x64-10 draws.
//
// Every workgroup is one wave of 64 lanes; all arithmetic is binary32.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pv_internal.h"

namespace pv {

// Vina-form weights: gauss1, gauss2, repulsion, hydrophobic, hydrogen bond.
constexpr float kW1 = -0.0356f, kW2 = -0.00516f, kW3 = 0.840f, kW4 = -0.0351f, kW5 = -0.587f;
constexpr float kCut2 = 64.0f;
constexpr float kPi = 3.14159265358979323846f;

// ---------------------------------------------------------------- wave helpers
// Cross-lane sums use DPP row permutations inside each 16-lane row and
// readlane across rows: a few VALU cycles instead of LDS round trips, and
// every lane ends with bit-identical results (the control flow that depends
// on them stays uniform).
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp0(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ float lane_f(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ int lane_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// sum over the 64 lanes, identical in every lane
__device__ __forceinline__ float wsum(float v)
{
    v += dpp0<0xB1>(v);   // quad_perm(1,0,3,2): lane ^ 1
    v += dpp0<0x4E>(v);   // quad_perm(2,3,0,1): lane ^ 2
    v += dpp0<0x141>(v);  // row_half_mirror: the other quad of each 8 lanes
    v += dpp0<0x140>(v);  // row_mirror: the other half of each row
    return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}

// sum over lanes 0..n-1 of v, where every lane from n up holds zero (n is
// wave-uniform): rows past the last non-zero one are not read
__device__ __forceinline__ float wsum_n(float v, int n)
{
    v += dpp0<0xB1>(v);
    v += dpp0<0x4E>(v);
    v += dpp0<0x141>(v);
    v += dpp0<0x140>(v);
    if (n <= 16) return lane_f(v, 0);
    if (n <= 32) return lane_f(v, 0) + lane_f(v, 16);
    return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}

// integer sum over the 64 lanes, identical in every lane
__device__ __forceinline__ int64_t wsum_i64(int64_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// inclusive prefix sum over the 64 lanes in lane order
__device__ __forceinline__ float wscan(float v)
{
    v += dpp0<0x111>(v);        // row_shr:1
    v += dpp0<0x112>(v);        // row_shr:2
    v += dpp0<0x114>(v);        // row_shr:4
    v += dpp0<0x118>(v);        // row_shr:8
    v += dpp0<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp0<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// the lane within the wave for the one-wave workgroups of the docking kernels
// (multi-wave kernels take threadIdx.x & (kWave - 1))
__device__ __forceinline__ int lane_id() { return threadIdx.x; }

// Synchronisation of a one-wave workgroup.  The LDS executes the requests of
// one wave in order, so ordering the compiler is enough: no wait for
// outstanding global loads (which may stay in flight across it).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}


// ---------------------------------------------------------------- Philox4x64-10
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t h0 = __umul64hi(M0, c[0]), l0 = M0 * c[0];
        uint64_t h1 = __umul64hi(M1, c[2]), l1 = M1 * c[2];
        uint64_t n0 = h1 ^ c[1] ^ k0, n2 = h0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = l1; c[2] = n2; c[3] = l0;
    }
}

__device__ __forceinline__ float u01(uint64_t w) { return (float)(uint32_t)(w >> 40) * 0x1p-24f; }

// counter = (block, step, chain, job), key = (seed, 0)
__device__ __forceinline__ uint64_t philox_word(uint64_t seed, int job, int chain, uint64_t step,
                                                uint64_t block, int word)
{
    uint64_t c[4] = {block, step, (uint64_t)chain, (uint64_t)job};
    philox4x64_10(c, seed, 0);
    return word == 0 ? c[0] : word == 1 ? c[1] : word == 2 ? c[2] : c[3];
}

// ---------------------------------------------------------------- small rotations
__device__ __forceinline__ void quat_mul(const float a[4], const float b[4], float o[4])
{
    float r0 = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    float r1 = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    float r2 = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    float r3 = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
}

__device__ __forceinline__ void rotvec_quat(float tx, float ty, float tz, float q[4])
{
    // (cos(a/2), sin(a/2)/a * theta); sin(a/2)/a -> 1/2 as a -> 0.  One
    // v_rsq gives both a = a^2 / a and 1 / a (hardware, ~1 ulp).
    const float a2 = tx * tx + ty * ty + tz * tz;
    const float inv = __builtin_amdgcn_rsqf(fmaxf(a2, 1e-30f));
    const float a = a2 * inv;
    float s, c;
    __sincosf(0.5f * a, &s, &c);
    const float k = a2 > 1e-30f ? s * inv : 0.5f;
    q[0] = c; q[1] = k * tx; q[2] = k * ty; q[3] = k * tz;
}

__device__ __forceinline__ void quat_normalize(float q[4])
{
    const float n = __builtin_amdgcn_rsqf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    q[0] *= n; q[1] *= n; q[2] *= n; q[3] *= n;
}

// ---------------------------------------------------------------- per-box grid view
struct BoxView {
    const float* maps;  // 8 maps of the box
    int nx, ny, nz;
    int64_t msz;
    float ox, oy, oz, h, inv_h, ex, ey, ez, kappa;
};

__device__ __forceinline__ BoxView box_view(const GridDev& g, int box)
{
    BoxView v;
    v.maps = g.maps + g.map_off[box];
    v.nx = g.dims[4 * box]; v.ny = g.dims[4 * box + 1]; v.nz = g.dims[4 * box + 2];
    v.msz = (int64_t)v.nx * v.ny * v.nz;
    const float* ge = g.geom + 8 * box;
    v.ox = ge[0]; v.oy = ge[1]; v.oz = ge[2]; v.h = ge[3]; v.inv_h = ge[4];
    v.ex = ge[5]; v.ey = ge[6]; v.ez = ge[7];
    v.kappa = g.kappa;
    return v;
}

// One axis of the lookup: fractional coordinate clamped to [0, n-1], cell
// i0 = min(floor f, n-2), the out-of-box penalty and whether the axis is
// clamped (its interpolant gradient is then zero).
__device__ __forceinline__ void axis_setup(float x, float o, float inv_h, float ext, int n, float kappa,
                                           int& i0, float& u, float& pen, float& dpen, bool& clamped)
{
    // no branches: at most one side is out (ext >= 0), so the penalty is the
    // sum of both sides' excess; a NaN coordinate is on neither side and
    // keeps its NaN in f
    const float rel = x - o;
    const bool lo = x < o, hi = rel > ext;
    pen = kappa * (fmaxf(o - x, 0.f) + fmaxf(rel - ext, 0.f));
    dpen = lo ? -kappa : (hi ? kappa : 0.f);
    const float f = lo ? 0.f : (hi ? (float)(n - 1) : rel * inv_h);
    clamped = lo || hi;
    int c = (int)floorf(f);
    c = max(0, min(c, n - 2));  // also keeps a NaN coordinate inside the map
    i0 = c;
    u = f - (float)c;
}

// Trilinear lookup in two halves: tri_issue computes the cell and starts the
// 8 corner loads; tri_finish interpolates (value, gradient, penalty) once
// they are needed, so other work can hide the memory latency in between.
struct TriLoad {
    float m[8];
    float ux, uy, uz, pen, dx, dy, dz;
    bool cx, cy, cz;
};

__device__ __forceinline__ void tri_issue(const BoxView& B, int t, float x, float y, float z, TriLoad& L)
{
    int ix, iy, iz;
    float px, py, pz;
    axis_setup(x, B.ox, B.inv_h, B.ex, B.nx, B.kappa, ix, L.ux, px, L.dx, L.cx);
    axis_setup(y, B.oy, B.inv_h, B.ey, B.ny, B.kappa, iy, L.uy, py, L.dy, L.cy);
    axis_setup(z, B.oz, B.inv_h, B.ez, B.nz, B.kappa, iz, L.uz, pz, L.dz, L.cz);
    L.pen = px + py + pz;
    // a box's 8 maps hold fewer than 8 x 2^24 points (checked when the grids
    // are built), so the corner offsets are 32-bit byte offsets from the
    // maps' base, formed with 24-bit multiplies
    const uint32_t nx = (uint32_t)B.nx, ny = (uint32_t)B.ny;
    const uint32_t e = __umul24((uint32_t)t, (uint32_t)B.msz) + __umul24(__umul24((uint32_t)iz, ny) + (uint32_t)iy, nx) +
                       (uint32_t)ix;
    const uint32_t o0 = e << 2, oy = nx << 2, oz = __umul24(nx, ny) << 2;
    const char* mb = (const char*)B.maps;
    const float* r0 = (const float*)(mb + o0);
    const float* r1 = (const float*)(mb + (o0 + oy));
    const float* r2 = (const float*)(mb + (o0 + oz));
    const float* r3 = (const float*)(mb + (o0 + oz + oy));
    L.m[0] = r0[0]; L.m[1] = r0[1];
    L.m[2] = r1[0]; L.m[3] = r1[1];
    L.m[4] = r2[0]; L.m[5] = r2[1];
    L.m[6] = r3[0]; L.m[7] = r3[1];
}

__device__ __forceinline__ float tri_finish(const BoxView& B, const TriLoad& L, float& gx, float& gy, float& gz)
{
    const float m000 = L.m[0], m100 = L.m[1], m010 = L.m[2], m110 = L.m[3];
    const float m001 = L.m[4], m101 = L.m[5], m011 = L.m[6], m111 = L.m[7];
    const float ux = L.ux, uy = L.uy, uz = L.uz;
    float a00 = m000 + ux * (m100 - m000), a10 = m010 + ux * (m110 - m010);
    float a01 = m001 + ux * (m101 - m001), a11 = m011 + ux * (m111 - m011);
    float b0 = a00 + uy * (a10 - a00), b1 = a01 + uy * (a11 - a01);
    float v = b0 + uz * (b1 - b0);
    // derivatives of the interpolant in the cell
    float d00 = m100 - m000, d10 = m110 - m010, d01 = m101 - m001, d11 = m111 - m011;
    float e0 = d00 + uy * (d10 - d00), e1 = d01 + uy * (d11 - d01);
    float dvx = e0 + uz * (e1 - e0);
    float dvy = (a10 - a00) + uz * ((a11 - a01) - (a10 - a00));
    float dvz = b1 - b0;
    gx = (L.cx ? 0.f : dvx * B.inv_h) + L.dx;
    gy = (L.cy ? 0.f : dvy * B.inv_h) + L.dy;
    gz = (L.cz ? 0.f : dvz * B.inv_h) + L.dz;
    return v + L.pen;
}

// trilinear value + gradient of map `t` at x, plus the penalty
__device__ __forceinline__ float trilinear(const BoxView& B, int t, float x, float y, float z, float& gx,
                                           float& gy, float& gz)
{
    TriLoad L;
    tri_issue(B, t, x, y, z, L);
    return tri_finish(B, L, gx, gy, gz);
}

// ---------------------------------------------------------------- LDS carving
// Pose slots hold [t(3), q(4), psi(T)] = up to 39 floats; 40 with padding.
constexpr int kSlot = 40;
enum { SLOT_X = 0, SLOT_XT = 1, SLOT_XA = 2, SLOT_CUR = 3, SLOT_BEST = 4, kNSlots = 5 };

struct Lds {
    char* base;        // start of the workgroup's dynamic LDS
    float* pose;       // [kNSlots][kSlot]
    float* frame;      // [kMaxFrag][12] frames, then [kMaxFrag] ancestor links / torsion derivatives
                       // (without the frames: the [kMaxFrag] torsion derivatives only)
    float4* pos;       // [ma + 1]; entry ma: a point far outside every box
    float4* frc;       // [max_atoms] dE/dx per atom, or NULL when nothing reads it back
    float* pre;        // [6][max_atoms]
    uint4* pairs;      // [max_pairs rounded up to kPairPass] pair records, slot layout (see stage_ligand)
    float* cp;         // [max_pairs rounded up to kWave] per-pair force coefficient, gather layout
    uint32_t* pw;      // [max_pairs rounded up to kWave] pair words, gather layout (padding: the far point)
    float4* fs;        // [max_ell + 1] pair forces in slot rows of n | 1 atoms (slot-major), then one
                       // write-only slot for the padding records, slot layout
    int ma;
};

// LDS byte address of a pointer into LDS, and back.
typedef __attribute__((address_space(3))) char lds_char;
__device__ __forceinline__ uint32_t lds_addr(const void* p)
{
    return (uint32_t)(uintptr_t)(const lds_char*)p;
}
template <typename V>
__device__ __forceinline__ __attribute__((address_space(3))) V* lds_ptr(uint32_t a)
{
    return (__attribute__((address_space(3))) V*)(uintptr_t)a;
}

// Pairs per pass of the pair loop (lanes x pairs per lane); the LDS pair
// records are padded to a multiple of it.
constexpr int kPairUnroll = 4;
constexpr int kPairPass = kPairUnroll * kWave;

__host__ __device__ inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Atom entries of the per-wave atom arrays (a multiple of 4 keeps every
// region 16-byte aligned).
__host__ __device__ inline int lds_atoms(int max_atoms) { return round_up(max_atoms < 1 ? 1 : max_atoms, 4); }

// Two layouts of the intra-force tables.  Slots (ligands of at most 64
// atoms, one atom per lane): the pair list sits in LDS, packed with the slots
// each pair owns in its two atoms' rows, beside the per-slot pair forces, so
// an atom's intra force is a stream of independent LDS reads.  Gather: the
// pair words and the per-pair coefficients live in LDS and the atom -> pair
// table is read from global memory (a small footprint, for large ligands or
// launches that need many resident waves).
//
// Optional regions: the per-atom forces (read back only by the score
// kernel's coordinate gradient) and the fragment frames (needed when atoms
// take their frames from LDS: two atoms per lane, and the output stage's
// pose positions; with one atom per lane the frames travel by ds_bpermute
// and only the torsion derivatives use the area).
struct LdsNeeds {
    bool slots, frc, frames;
    bool pw;   // gather layout: the pair words in LDS too (one atom per lane), else read from global memory
};

__host__ __device__ inline int lds_bytes(int max_atoms, int max_pairs, int max_ell, LdsNeeds nd)
{
    const int ma = lds_atoms(max_atoms);
    int b = kNSlots * kSlot * 4 + (ma + 1) * 16 + 6 * ma * 4;
    b += nd.frames ? kMaxFrag * 13 * 4 + 12 : round_up(kMaxFrag, 4) * 4;
    if (nd.frc) b += ma * 16;
    if (nd.slots) b += round_up(max_pairs < 1 ? 1 : max_pairs, kPairPass) * 16 + (max_ell + 1) * 16;
    else b += (nd.pw ? 2 : 1) * round_up(max_pairs + 1, kWave) * 4;
    return b;
}

__device__ __forceinline__ Lds carve(char* base, int max_atoms, int max_pairs, int max_ell, LdsNeeds nd)
{
    Lds s;
    const int ma = lds_atoms(max_atoms);
    char* p = base;
    s.base = base;
    s.pos = (float4*)p; p += (ma + 1) * 16;
    s.pose = (float*)p; p += kNSlots * kSlot * 4;
    s.pre = (float*)p; p += 6 * ma * 4;
    s.frc = nullptr;
    if (nd.frc) { s.frc = (float4*)p; p += ma * 16; }
    s.frame = (float*)p; p += nd.frames ? kMaxFrag * 13 * 4 + 12 : round_up(kMaxFrag, 4) * 4;
    s.pairs = nullptr; s.fs = nullptr; s.cp = nullptr; s.pw = nullptr;
    if (nd.slots) {
        s.pairs = (uint4*)p; p += round_up(max_pairs < 1 ? 1 : max_pairs, kPairPass) * 16;
        s.fs = (float4*)p;
    } else {
        const int pp = round_up(max_pairs + 1, kWave);
        s.cp = (float*)p; p += pp * 4;
        if (nd.pw) s.pw = (uint32_t*)p;
    }
    s.ma = ma;
    return s;
}

// Torsion derivatives in LDS: after the frames (and their links) when the
// frames are stored, else at the start of the frame area.
__device__ __forceinline__ float* dpsi_area(const Lds& S, bool frames) { return frames ? S.frame + 12 * kMaxFrag : S.frame; }

// The regions a kernel's LDS holds: per-atom forces for the score kernel's
// coordinate gradient; frames for two atoms per lane and the output stage;
// the pair words for one atom per lane on the gather layout (with two atoms
// per lane the pair lists are long and the words stay in global memory, so
// that LDS does not cut the resident waves).
constexpr int kKindOutput = 3;
__host__ __device__ inline LdsNeeds kernel_needs(int kind, int A, bool slots)
{
    return LdsNeeds{slots, kind == kKindScore, A > 1 || kind == kKindOutput, !slots && A == 1};
}

// Least value over all surface distances of a pair's energy, by class (the
// Vina terms above: plain at d = 0.003, hydrophobic at d = 0.003, hydrogen
// bond at d = -0.466), rounded down in the fourth digit.
constexpr float kPairMin0 = -0.03615f, kPairMin1 = -0.07125f, kPairMin2 = -0.22356f;

// ---------------------------------------------------------------- staged ligand
// Topology lives in registers: atoms blocked A per lane (atom = lane*A + a),
// fragments one per lane, and for lane 6+k the fragment of torsion k.
template <int A, bool SL>
struct Topo {
    int n, nf, nt, np, rounds, lig, ell_w, fs_stride;
    float anc_x, anc_y, anc_z, rot_scale;
    float4 ref[A];
    int f_parent, f_tors, f_child, f_a0, f_end;
    uint64_t links;   // the ancestor a fragment lane composes with in each pointer-doubling round, 6 bits per
                      // round (63: none): fragments 0..32 and up to 6 rounds
    float ax, ay, az, cx, cy, cz;
    int dof_frag;
    float lb;   // a lower bound of the intra energy: the sum over the pairs of their class's least pair energy
    const uint32_t* gpairs;   // pair list and atom -> pair table in global
    const uint32_t* gell;     // memory (read from there when A > 1)
};

template <int A, bool SL>
__device__ void stage_ligand(Topo<A, SL>& T, const LigDev& L, int lig, const Lds& S)
{
    const int l = lane_id();
    const DevLig d = L.ligs[lig];
    T.lig = lig;
    T.n = d.n_atoms; T.nf = d.n_frag; T.nt = d.n_tors; T.np = d.n_pairs; T.rounds = d.rounds;
    T.ell_w = d.ell_w;
    // slot rows of an odd number of float4 (one per atom): the row reads of
    // the gather are contiguous, and the slots of one atom fall in different
    // LDS banks
    T.fs_stride = T.n | 1;
    T.anc_x = d.anchor[0]; T.anc_y = d.anchor[1]; T.anc_z = d.anchor[2]; T.rot_scale = d.rot_amp_scale;
#pragma unroll
    for (int a = 0; a < A; ++a) {
        int i = l * A + a;
        T.ref[a] = i < T.n ? L.atoms[d.atom_base + i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (l < T.nf) {
        const DevFrag F = L.frags[d.frag_base + l];
        T.f_parent = F.parent; T.f_tors = F.tors; T.f_child = F.child_atom; T.f_a0 = F.a0; T.f_end = F.sub_end;
        T.ax = F.axis[0]; T.ay = F.axis[1]; T.az = F.axis[2];
        T.cx = F.xc[0]; T.cy = F.xc[1]; T.cz = F.xc[2];
    } else {
        T.f_parent = -1; T.f_tors = -1; T.f_child = 0; T.f_a0 = 0; T.f_end = 0;
        T.ax = T.ay = T.az = T.cx = T.cy = T.cz = 0.f;
    }
    T.dof_frag = (l >= 6 && l < 6 + T.nt) ? (int)L.tors_frag[d.tors_base + l - 6] : 0;
    {
        // the links do not depend on the pose: jumped once here (a lane
        // with an ancestor takes that ancestor's link after each round)
        static_assert(kMaxFrag <= 63, "a link holds a fragment index below 63");
        int anc = (l >= 1 && l < T.nf) ? T.f_parent : -1;
        T.links = 0;
        for (int r = 0; r < T.rounds; ++r) {
            T.links |= (uint64_t)(anc >= 0 ? anc : 63) << (6 * r);
            const int panc = __builtin_amdgcn_ds_bpermute((anc >= 0 ? anc : l) << 2, anc);
            if (anc >= 0) anc = panc;
        }
    }
    T.gpairs = L.pairs + d.pair_base;
    T.gell = L.ell + d.ell_base;
    {
        // least pair energy of each class (plain, hydrophobic, hydrogen
        // bond) over all distances, rounded down; a pair past the cutoff
        // adds 0, which is above them
        float lbl = 0.f;
        for (int p = l; p < T.np; p += kWave) {
            const uint32_t c = T.gpairs[p] >> 24;
            lbl += c == 0 ? kPairMin0 : (c == 1 ? kPairMin1 : kPairMin2);
        }
        T.lb = wsum(lbl);
    }
    if (l == 0) S.pos[S.ma] = make_float4(1e18f, 1e18f, 1e18f, 0.f);
    if (SL) {
        // Pair record, everything the pair loop needs without decoding:
        //   x: LDS byte addresses of both positions (i | j << 16; S.pos opens
        //      the LDS, so both fit) | class << 30
        //   y, z: LDS byte addresses of the pair's force slots in the rows of
        //         i and of j (slot * row stride + atom)
        //   w: the radius sum 3.4 + 0.1 rk (bits)
        // Records past the last pair fill the final pass: their first atom is
        // the far point, so they fall outside the cutoff, and both their
        // slots are the write-only one past the rows.
        const uint32_t* ps = L.pslot + d.pair_base;
        const uint32_t ns = (uint32_t)T.fs_stride;
        const int nfs = T.ell_w * T.fs_stride;
        const uint32_t fs0 = lds_addr(S.fs), pos0 = lds_addr(S.pos);
        const int npad = round_up(T.np < 1 ? 1 : T.np, kPairPass);
        for (int p = l; p < npad; p += kWave) {
            uint4 r;
            if (p < T.np) {
                const uint32_t pk = T.gpairs[p], sl = ps[p];
                const uint32_t i = pk & 0xff, j = (pk >> 8) & 0xff;
                r.x = (pos0 + (i << 4)) | (pos0 + (j << 4)) << 16 | ((pk >> 24) << 30);
                r.y = fs0 + (((sl & 0xffff) * ns + i) << 4);
                r.z = fs0 + (((sl >> 16) * ns + j) << 4);
                r.w = __float_as_uint(fmaf((float)((pk >> 16) & 7u), 0.1f, 3.4f));
            } else {
                r.x = pos0 + ((uint32_t)S.ma << 4);
                r.y = r.z = fs0 + ((uint32_t)nfs << 4);
                r.w = __float_as_uint(3.4f);
            }
            S.pairs[p] = r;
        }
        for (int k = l; k < nfs; k += kWave) S.fs[k] = make_float4(0.f, 0.f, 0.f, 0.f);   // padding stays zero
    } else {
        // one atom per lane: pair words up to a whole pass of 64 in LDS; the padding pairs join the far
        // point to atom 0, so they fall outside the cutoff and store c = 0
        // (which also serves the atom -> pair table's padding entries, p = np)
        if (A == 1) {
            // eight loads per lane in flight before their stores
            const int npad = round_up(T.np + 1, kWave);
            for (int p0 = l; p0 < npad; p0 += 8 * kWave) {
                uint32_t w[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int p = p0 + q * kWave;
                    w[q] = p < T.np ? T.gpairs[p] : (uint32_t)S.ma;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (p0 + q * kWave < npad) S.pw[p0 + q * kWave] = w[q];
            }
        }
        if (l == 0) S.cp[T.np] = 0.f;   // not written by the pair loop when np is a multiple of 64
    }
    wave_sync();
}

// ---------------------------------------------------------------- evaluation
struct Eval {
    float e, e_inter, e_intra;
    float g;          // this lane's tangent component (lane < 6 + T)
    int pairs_in;     // this lane's intra pairs inside the cutoff
    bool outside;     // some atom lies outside the box (its lookup was clamped)
    bool bounded;     // a trial decided by its map energy and the intra bound (no pair loop)
};

// Frame of every fragment: x = R X + b on reference coordinates.  Lane f
// starts from its local map (the root's pose map, or the rotation by psi
// about its torsion axis) and composes with its ancestors by pointer
// doubling; after `rounds` rounds every frame is world-absolute.
template <int A, bool SL>
__device__ __forceinline__ void frames(const Topo<A, SL>& T, const Lds& S, const float* pose, float R[9], float b[3])
{
    const int l = lane_id();
    // Local map of every fragment lane, one formula for the root and the
    // torsions: R = I + [s]x + w w^T - |w|^2 I, b = p - R a.
    //   root:     unit q = (qw, v): s = 2 qw v, w = sqrt(2) v; p = t, a = anchor
    //   torsion:  angle psi about unit axis u through c: with h = psi / 2,
    //             s = 2 sin h cos h u, w = sqrt(2) sin h u; p = a = c
    const float qw = pose[3], qx = pose[4], qy = pose[5], qz = pose[6];
    const float qi = __builtin_amdgcn_rsqf(qw * qw + qx * qx + qy * qy + qz * qz);
    const bool root = l == 0;
    float sh, ch;
    __sincosf(0.5f * pose[7 + (root ? 0 : T.f_tors)], &sh, &ch);
    const float ux = root ? qx * qi : T.ax, uy = root ? qy * qi : T.ay, uz = root ? qz * qi : T.az;
    const float k1 = root ? 2.f * qw * qi : 2.f * sh * ch;
    const float k2 = root ? 1.41421356f : 1.41421356f * sh;
    const float sx = k1 * ux, sy = k1 * uy, sz = k1 * uz;
    const float wx = k2 * ux, wy = k2 * uy, wz = k2 * uz;
    const float c0 = 1.f - (wx * wx + wy * wy + wz * wz);
    R[0] = c0 + wx * wx; R[1] = wx * wy - sz;  R[2] = wx * wz + sy;
    R[3] = wy * wx + sz; R[4] = c0 + wy * wy;  R[5] = wy * wz - sx;
    R[6] = wz * wx - sy; R[7] = wz * wy + sx;  R[8] = c0 + wz * wz;
    const float px = root ? pose[0] : T.cx, py = root ? pose[1] : T.cy, pz = root ? pose[2] : T.cz;
    const float ax = root ? T.anc_x : T.cx, ay = root ? T.anc_y : T.cy, az = root ? T.anc_z : T.cz;
    b[0] = px - (R[0] * ax + R[1] * ay + R[2] * az);
    b[1] = py - (R[3] * ax + R[4] * ay + R[5] * az);
    b[2] = pz - (R[6] * ax + R[7] * ay + R[8] * az);
    // pointer doubling across lanes: every round each fragment fetches the
    // partial frame of its ancestor of that round (links jumped at staging)
    // straight from that lane's registers (ds_bpermute, all lanes taking
    // part), then composes; a lane without an ancestor fetches its own
    // values and keeps its frame
    for (int r = 0; r < T.rounds; ++r) {
        const int anc = (int)(T.links >> (6 * r)) & 63;
        const int src = (anc != 63 ? anc : l) << 2;
        float P[9], pb[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) P[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(R[k])));
#pragma unroll
        for (int k = 0; k < 3; ++k) pb[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(b[k])));
        if (anc != 63) {
            float N[9], nb[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    N[3 * i + j] = P[3 * i] * R[j] + P[3 * i + 1] * R[3 + j] + P[3 * i + 2] * R[6 + j];
                nb[i] = P[3 * i] * b[0] + P[3 * i + 1] * b[1] + P[3 * i + 2] * b[2] + pb[i];
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) R[k] = N[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) b[k] = nb[k];
        }
    }
}

// Intra pairs, lanes over pairs, kPairUnroll pairs per lane and pass: every
// load of a pass (pair records, then both positions) is issued before any of
// its arithmetic, so the LDS latency is paid once per pass.  Per pair, with d
// the surface distance and inside 8 A: the gauss, repulsion, hydrophobic and
// hydrogen-bond terms of the Vina form and the force coefficient
// c = (dphi/dr) / r.  Pairs are grouped by interaction class, so a whole
// 64-pair chunk usually has no hydrophobic or hydrogen-bond weight and skips
// those terms on a wave-uniform branch.  With the tables in LDS each pair
// writes +f / -f into its slots of the two atoms' rows (the padded records
// make every pass full, with no per-lane guard); otherwise it stores c for
// the table gather.  No atomics either way.  Returns this lane's energy; adds
// this lane's pairs inside the cutoff to cnt.
typedef float f3v __attribute__((ext_vector_type(3)));
constexpr float kLog2e = 1.4426950408889634f;

// One pass of U pairs per lane starting at pair p0 (this lane's first);
// adds this lane's energy to e and its pairs inside the cutoff to cnt.
template <int A, bool SL, int U>
__device__ __forceinline__ void pair_pass(const Topo<A, SL>& T, const Lds& S, int p0, float& e, int& cnt,
                                          const uint32_t* words = nullptr)
{
    const uint32_t pos0 = lds_addr(S.pos);
    // position addresses; slot addresses; radius sum bits (slots) or
    // the pair word's upper half, radius-sum code | class << 8 (gather)
    uint32_t ai[U], aj[U], ya[U], za[U], rc[U];
    bool v[U];
    float4 xi[U], xj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = p0 + u * kWave;
        if (SL) {
            const uint4 w = S.pairs[p];
            ai[u] = w.x & 0xffffu; aj[u] = w.x >> 16;   // the class sits above bit 29: kept for the test
            ya[u] = w.y; za[u] = w.z; rc[u] = w.w;
            v[u] = true;
        } else {
            // LDS pair words are padded to whole passes of 64 with far-point
            // pairs; with two atoms per lane the caller brings the words
            // from global memory (a lane past the end holds pair 0 and
            // discards it)
            uint32_t g;
            if (A == 1) {
                g = S.pw[p];
                v[u] = true;
            } else {
                v[u] = p < T.np;
                g = words[u];
            }
            ai[u] = pos0 + ((g & 0xffu) << 4); aj[u] = pos0 + (((g >> 8) & 0xffu) << 4);
            rc[u] = g >> 16;
            ya[u] = za[u] = 0u;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        xi[u] = *(const float4*)lds_ptr<const float4>(ai[u]);
        xj[u] = *(const float4*)lds_ptr<const float4>(SL ? aj[u] & 0x3fffu : aj[u]);
    }
    float dx[U], dy[U], dz[U], d[U], en[U], de[U], rinv[U];
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        dx[u] = xi[u].x - xj[u].x; dy[u] = xi[u].y - xj[u].y; dz[u] = xi[u].z - xj[u].z;
        const float r2 = dx[u] * dx[u] + dy[u] * dy[u] + dz[u] * dz[u];
        in[u] = v[u] && r2 < kCut2;
        // one v_rsq_f32: r = r2 / sqrt(r2) and c = de / r = de * rsq; a
        // zero distance gets a tiny finite r and its zero direction
        // zeroes the force
        const float r2c = fmaxf(r2, 1e-12f);
        rinv[u] = __builtin_amdgcn_rsqf(r2c);
        const float rs = SL ? __uint_as_float(rc[u]) : fmaf((float)(rc[u] & 0xffu), 0.1f, 3.4f);
        const float dd = r2c * rinv[u] - rs;
        d[u] = dd;
        // exp(-(d/0.5)^2) and exp(-((d-3)/2)^2), the second exponent
        // expanded around d^2 so both share it: c (d-3)^2 = c d^2 - 6c d + 9c
        const float d2 = dd * dd;
        const float g1 = __builtin_amdgcn_exp2f(d2 * (-4.f * kLog2e));
        constexpr float c2 = -0.25f * kLog2e;
        const float g2 = __builtin_amdgcn_exp2f(fmaf(d2, c2, fmaf(dd, -6.f * c2, 9.f * c2)));
        const float dn = fminf(dd, 0.f);                                             // repulsion d^2, d < 0
        en[u] = fmaf(kW1, g1, fmaf(kW2, g2, kW3 * (dn * dn)));
        constexpr float k2 = -0.5f * kW2;                                            // d/dd of the second: k2 (d-3)
        de[u] = fmaf(g1, dd * (-8.f * kW1), fmaf(g2, fmaf(dd, k2, -3.f * k2), dn * (2.f * kW3)));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        // class 1 (both hydrophobic) adds the hydrophobic term, class 2
        // (donor with acceptor) the hydrogen-bond term
        const uint32_t cls = SL ? aj[u] >> 14 : rc[u] >> 8;
        if (__ballot(cls != 0u)) {
            const float wy = cls == 1u ? kW4 : 0.f, wz = cls == 2u ? kW5 : 0.f;
            const float dd = d[u];
            const float hv = fminf(fmaxf(1.5f - dd, 0.f), 1.f);            // 1 below 0.5, 0 above 1.5
            const float bv = fminf(fmaxf(dd * -(1.f / 0.7f), 0.f), 1.f);   // 1 below -0.7, 0 above 0
            en[u] = fmaf(wy, hv, fmaf(wz, bv, en[u]));
            const float hs = (dd >= 0.5f && dd < 1.5f) ? -wy : 0.f;
            const float bs = (dd >= -0.7f && dd < 0.f) ? wz * -(1.f / 0.7f) : 0.f;
            de[u] += hs + bs;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        e += in[u] ? en[u] : 0.f;
        cnt += in[u] ? 1 : 0;
        const float c = in[u] ? de[u] * rinv[u] : 0.f;
        if (SL) {
            // 12-byte writes (ds_write_b96) into the 16-byte slots; the
            // gather reads x, y, z
            const float fx = c * dx[u], fy = c * dy[u], fz = c * dz[u];
            *(f3v*)lds_ptr<f3v>(ya[u]) = f3v{fx, fy, fz};
            *(f3v*)lds_ptr<f3v>(za[u]) = f3v{-fx, -fy, -fz};
        } else if (v[u]) {
            S.cp[p0 + u * kWave] = c;
        }
    }
}

// Intra pairs, lanes over pairs: whole passes of kPairUnroll pairs per lane
// (every load of a pass issued before any of its arithmetic, so the LDS
// latency is paid once per pass), then, on the gather layout with one atom
// per lane, whole passes of two pairs per lane and passes of one over the
// rest, so at most 63 padding pairs are evaluated.
// Per pair, with d the surface distance and inside 8 A: the gauss,
// repulsion, hydrophobic and hydrogen-bond terms of the Vina form and the
// force coefficient c = (dphi/dr) / r.  Pairs are grouped by interaction
// class, so a whole 64-pair chunk usually has no hydrophobic or
// hydrogen-bond weight and skips those terms on a wave-uniform branch.  With
// the slot layout each pair writes +f / -f into its slots of the two atoms'
// rows (records padded to whole passes, no per-lane guard); otherwise it
// stores c for the table gather.  No atomics either way.  Returns this
// lane's energy; adds this lane's pairs inside the cutoff to cnt.
template <int A, bool SL>
__device__ __forceinline__ float pair_loop(const Topo<A, SL>& T, const Lds& S, int& cnt)
{
    const int l = lane_id();
    const int np = T.np;
    float e = 0.f;
    int p0 = l;
    if (SL) {
        for (; p0 - l < np; p0 += kPairPass) pair_pass<A, SL, kPairUnroll>(T, S, p0, e, cnt);
    } else {
        if (A > 1) {
            // two atoms per lane (ligands of 65 to 128 atoms, long pair
            // lists): whole passes only; the pair words come from global
            // memory, each pass's loaded during the pass before (a lane past
            // the end reads pair 0, np >= 1 here, and discards it)
            uint32_t w[kPairUnroll], nw[kPairUnroll];
            if (np > 0) {
#pragma unroll
                for (int u = 0; u < kPairUnroll; ++u) {
                    const int p = p0 + u * kWave;
                    w[u] = T.gpairs[p < np ? p : 0];
                }
            }
            for (; p0 - l < np; p0 += kPairPass) {
#pragma unroll
                for (int u = 0; u < kPairUnroll; ++u) {
                    const int p = p0 + kPairPass + u * kWave;
                    nw[u] = T.gpairs[p < np ? p : 0];
                }
                pair_pass<A, SL, kPairUnroll>(T, S, p0, e, cnt, w);
#pragma unroll
                for (int u = 0; u < kPairUnroll; ++u) w[u] = nw[u];
            }
        } else {
            for (; p0 - l + kPairPass <= np; p0 += kPairPass) pair_pass<A, SL, kPairUnroll>(T, S, p0, e, cnt);
            for (; p0 - l + 2 * kWave <= np; p0 += 2 * kWave) pair_pass<A, SL, 2>(T, S, p0, e, cnt);
            for (; p0 - l < np; p0 += kWave) pair_pass<A, SL, 1>(T, S, p0, e, cnt);
        }
    }
    return e;
}

// dE/dx_i of the intra term.  LDS tables: the sum of atom i's row of pair
// forces (independent reads, rows padded to a multiple of four with zeros).
// Global tables: sum over the pairs holding atom i of c_p (x_i - x_j); an
// entry holds p in its low half and j's byte offset in S.pos in its high half.
// row loads of the global atom -> pair table issued together by the gather:
// the table sits in L2, so a row walked one load at a time pays one L2
// round trip per four entries
constexpr int kGatherChunk = 8;

template <int A, bool SL>
__device__ __forceinline__ void gather_pair_forces(const Topo<A, SL>& T, const Lds& S, int i, float4 xi, float& gx,
                                                   float& gy, float& gz)
{
    if (SL) {
        // eight independent reads in flight per group (rows are padded to a
        // multiple of four, so at most one group of four is left)
        const float4* row = S.fs + i;
        const int ns = T.fs_stride;
        int k = 0;
        for (; k + 8 <= T.ell_w; k += 8) {
            float4 f[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) f[u] = row[(k + u) * ns];
#pragma unroll
            for (int u = 0; u < 8; ++u) { gx += f[u].x; gy += f[u].y; gz += f[u].z; }
        }
        if (k < T.ell_w) {
            float4 f[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) f[u] = row[(k + u) * ns];
#pragma unroll
            for (int u = 0; u < 4; ++u) { gx += f[u].x; gy += f[u].y; gz += f[u].z; }
        }
        return;
    }
    // the atom's row is contiguous ([n][ell_w], ell_w a multiple of four):
    // one 16-byte load per four entries, at an unsigned 32-bit offset from
    // the table's base (a scalar base plus one vector offset)
    // up to kGatherChunk loads of the row are issued before any is used, so
    // a row of at most 4 * kGatherChunk entries pays one load latency
    const char* row = (const char*)T.gell + (uint32_t)(i * T.ell_w * 4);
    for (int k0 = 0; k0 < T.ell_w; k0 += 4 * kGatherChunk) {
        uint4 e4[kGatherChunk];
#pragma unroll
        for (int q = 0; q < kGatherChunk; ++q)
            if (k0 + 4 * q < T.ell_w) e4[q] = *(const uint4*)(row + (uint32_t)((k0 + 4 * q) * 4));
#pragma unroll
        for (int q = 0; q < kGatherChunk; ++q) {
            if (k0 + 4 * q >= T.ell_w) break;
            const uint32_t e[4] = {e4[q].x, e4[q].y, e4[q].z, e4[q].w};
            float c[4];
            float4 xj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = S.cp[e[u] & 0xffff];
                xj[u] = *(const float4*)((const char*)S.pos + (e[u] >> 16));
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                gx += c[u] * (xi.x - xj[u].x);
                gy += c[u] * (xi.y - xj[u].y);
                gz += c[u] * (xi.z - xj[u].z);
            }
        }
    }
}

// World position of one atom from its reference record (x, y, z, type |
// fragment << 8) and its fragment's frame in LDS.
__device__ __forceinline__ float4 atom_position(float4 ref, const Lds& S)
{
    const int f = __float_as_uint(ref.w) >> 8;
    const float4* fr = (const float4*)(S.frame + 12 * f);
    const float4 r0 = fr[0], r1 = fr[1], r2 = fr[2];
    const float x = r0.x * ref.x + r0.y * ref.y + r0.z * ref.z + r2.y;
    const float y = r0.w * ref.x + r1.x * ref.y + r1.y * ref.z + r2.z;
    const float z = r1.z * ref.x + r1.w * ref.y + r2.x * ref.z + r2.w;
    return make_float4(x, y, z, 0.f);
}

// Score and tangent gradient of the pose in `pose` (an LDS slot).  Leaves
// atom positions in S.pos and dE/dx in S.frc.  When the energy exceeds
// e_limit (a line-search trial that fails the sufficient-decrease test,
// whose gradient nobody reads) it returns after the energy, with g = 0 and
// S.frc not written.  use_bound lets such a trial try the intra lower bound
// before its pair loop.
template <int A, bool SL>
__device__ Eval evaluate(const Topo<A, SL>& T, const BoxView& B, const Lds& S, const float* pose,
                         float e_limit = __builtin_inff(), bool use_bound = true)
{
    const int l = lane_id();
    Eval out;
    float R[9], b[3];
    frames(T, S, pose, R, b);
    // the world axis of this fragment lane's torsion, the one use of the
    // frame after the atom positions (so R and b need not stay live)
    const float awx = R[0] * T.ax + R[1] * T.ay + R[2] * T.az;
    const float awy = R[3] * T.ax + R[4] * T.ay + R[5] * T.az;
    const float awz = R[6] * T.ax + R[7] * T.ay + R[8] * T.az;
    if (A > 1) {
        if (l < T.nf) {
            float* fr = S.frame + 12 * l;
#pragma unroll
            for (int k = 0; k < 9; ++k) fr[k] = R[k];
            fr[9] = b[0]; fr[10] = b[1]; fr[11] = b[2];
        }
        wave_sync();
    }
    float e_in = 0.f;
    float4 X4[A];
    float G[A][3];
    TriLoad TL[A];
    if (A == 1) {
        // one atom per lane: its fragment's frame straight from that lane
        const int src = (int)(__float_as_uint(T.ref[0].w) >> 8) << 2;
        float P[9], pb[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) P[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(R[k])));
#pragma unroll
        for (int k = 0; k < 3; ++k) pb[k] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(b[k])));
        const float4 rf = T.ref[0];
        X4[0] = make_float4(P[0] * rf.x + P[1] * rf.y + P[2] * rf.z + pb[0],
                            P[3] * rf.x + P[4] * rf.y + P[5] * rf.z + pb[1],
                            P[6] * rf.x + P[7] * rf.y + P[8] * rf.z + pb[2], 0.f);
        G[0][0] = G[0][1] = G[0][2] = 0.f;
        if (l < T.n) {
            S.pos[l] = X4[0];
            tri_issue(B, __float_as_uint(rf.w) & 0xff, X4[0].x, X4[0].y, X4[0].z, TL[0]);
        } else {
            X4[0] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    } else {
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const int i = l * A + a;
            X4[a] = make_float4(0.f, 0.f, 0.f, 0.f);
            G[a][0] = G[a][1] = G[a][2] = 0.f;
            if (i < T.n) {
                X4[a] = atom_position(T.ref[a], S);
                S.pos[i] = X4[a];
            }
        }
    }
    wave_sync();
    // A line-search trial whose map energy plus the intra lower bound is
    // already above its sufficient-decrease bound is rejected by the full
    // energy too: it stops before the pair loop (a margin covers rounding).
    // The slot form runs few waves per SIMD, where ending the map loads before
    // the pair loop costs more latency than the skipped trials save: it
    // always runs both.
    const bool bound = !SL && use_bound && e_limit < 3.0e38f;   // wave-uniform
    bool outl = false, map_done = false;
    if (bound) {
        if (A > 1) {
#pragma unroll
            for (int a = 0; a < A; ++a)
                if (l * A + a < T.n)
                    tri_issue(B, __float_as_uint(T.ref[a].w) & 0xff, X4[a].x, X4[a].y, X4[a].z, TL[a]);
        }
#pragma unroll
        for (int a = 0; a < A; ++a)
            if (l * A + a < T.n) {
                e_in += tri_finish(B, TL[a], G[a][0], G[a][1], G[a][2]);
                outl = outl || TL[a].cx || TL[a].cy || TL[a].cz;
            }
        out.e_inter = wsum(e_in);
        map_done = true;
        if (out.e_inter + T.lb > e_limit + 1e-3f + 1e-4f * (fabsf(out.e_inter) + fabsf(T.lb))) {
            out.e_intra = T.lb;
            out.e = out.e_inter + T.lb;
            out.pairs_in = 0;
            out.outside = __ballot(outl) != 0;
            out.bounded = true;
            out.g = 0.f;
            wave_sync();
            return out;
        }
        // the map forces wait in the scan area (unused until the scans), so
        // no registers are held across the pair loop
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const int i = l * A + a;
            if (i < T.n) { S.pre[i] = G[a][0]; S.pre[S.ma + i] = G[a][1]; S.pre[2 * S.ma + i] = G[a][2]; }
        }
    }
    int cnt = 0;
    const float e_ia = pair_loop(T, S, cnt);   // hides the map loads (one atom per lane)
    // the energy sums start here, so their cross-lane steps overlap the
    // force gather and the scans below
    out.e_intra = wsum(e_ia);
    wave_sync();
    if (!map_done) {
        if (A > 1) {
            // two atoms per lane: the map loads start only now, since holding
            // both lookups across the pair loop would cost a resident wave
#pragma unroll
            for (int a = 0; a < A; ++a)
                if (l * A + a < T.n)
                    tri_issue(B, __float_as_uint(T.ref[a].w) & 0xff, X4[a].x, X4[a].y, X4[a].z, TL[a]);
        }
#pragma unroll
        for (int a = 0; a < A; ++a)
            if (l * A + a < T.n) {
                e_in += tri_finish(B, TL[a], G[a][0], G[a][1], G[a][2]);
                outl = outl || TL[a].cx || TL[a].cy || TL[a].cz;
            }
        out.e_inter = wsum(e_in);
    } else {
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const int i = l * A + a;
            if (i < T.n) { G[a][0] = S.pre[i]; G[a][1] = S.pre[S.ma + i]; G[a][2] = S.pre[2 * S.ma + i]; }
        }
    }
    out.outside = __ballot(outl) != 0;
    out.bounded = false;
    out.e = out.e_inter + out.e_intra;
    out.pairs_in = cnt;
    if (out.e > e_limit) {    // wave-uniform
        out.g = 0.f;
        wave_sync();
        return out;
    }
#pragma unroll
    for (int a = 0; a < A; ++a)
        if (l * A + a < T.n) gather_pair_forces(T, S, l * A + a, X4[a], G[a][0], G[a][1], G[a][2]);
    // per-atom force (inter + intra) and torque about t, blocked scan over atoms
    const float tx = pose[0], ty = pose[1], tz = pose[2];
    float v[A][6];
    float run[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < A; ++a) {
        const int i = l * A + a;
        float rx = 0, ry = 0, rz = 0;
        if (i < T.n) {
            if (S.frc) S.frc[i] = make_float4(G[a][0], G[a][1], G[a][2], 0.f);
            rx = X4[a].x - tx; ry = X4[a].y - ty; rz = X4[a].z - tz;
        }
        run[0] += G[a][0]; run[1] += G[a][1]; run[2] += G[a][2];
        run[3] += ry * G[a][2] - rz * G[a][1];
        run[4] += rz * G[a][0] - rx * G[a][2];
        run[5] += rx * G[a][1] - ry * G[a][0];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[a][c] = run[c];
    }
    float incl[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) incl[c] = wscan(run[c]);
    // atom i's prefix: lane i's inclusive scan (one atom per lane), else the
    // lane's exclusive scan plus its running sum up to the atom
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        if (A == 1) {
            if (l < T.n) S.pre[c * S.ma + l] = incl[c];
        } else {
            const float excl = incl[c] - run[c];
#pragma unroll
            for (int a = 0; a < A; ++a) {
                const int i = l * A + a;
                if (i < T.n) S.pre[c * S.ma + i] = excl + v[a][c];
            }
        }
    }
    wave_sync();
    // torsion derivative: world axis . sum over the moved atoms of (x - x_c) x G
    float dpsi = 0.f;
    if (l >= 1 && l < T.nf) {
        const int e = T.f_end - 1, s0 = T.f_a0 - 1;
        float Sg[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) Sg[c] = S.pre[c * S.ma + e] - S.pre[c * S.ma + s0];
        const float4 pc = S.pos[T.f_child];
        const float cx = pc.x - tx, cy = pc.y - ty, cz = pc.z - tz;
        const float mx = Sg[3] - (cy * Sg[2] - cz * Sg[1]);
        const float my = Sg[4] - (cz * Sg[0] - cx * Sg[2]);
        const float mz = Sg[5] - (cx * Sg[1] - cy * Sg[0]);
        dpsi = awx * mx + awy * my + awz * mz;
    }
    float* dps = dpsi_area(S, A > 1);
    if (l >= 1 && l < T.nf) dps[l] = dpsi;
    wave_sync();
    const int last = T.n - 1;
    float g = 0.f;
    if (l < 6) g = S.pre[l * S.ma + last];
    else if (l < 6 + T.nt) g = dps[T.dof_frag];
    out.g = g;
    wave_sync();
    return out;
}

// Score on given coordinates already in S.pos: forces in S.frc.
template <int A, bool SL>
__device__ Eval evaluate_xyz(const Topo<A, SL>& T, const BoxView& B, const Lds& S)
{
    const int l = lane_id();
    Eval out;
    float e_in = 0.f;
    int cnt = 0;
    const float e_ia = pair_loop(T, S, cnt);
    wave_sync();
#pragma unroll
    for (int a = 0; a < A; ++a) {
        const int i = l * A + a;
        if (i < T.n) {
            const int ty = __float_as_uint(T.ref[a].w) & 0xff;
            const float4 p = S.pos[i];
            float gx, gy, gz;
            e_in += trilinear(B, ty, p.x, p.y, p.z, gx, gy, gz);
            gather_pair_forces(T, S, i, p, gx, gy, gz);
            if (S.frc) S.frc[i] = make_float4(gx, gy, gz, 0.f);
        }
    }
    wave_sync();
    out.g = 0.f;
    out.outside = false;
    out.bounded = false;
    out.e_inter = wsum(e_in);
    out.e_intra = wsum(e_ia);
    out.e = out.e_inter + out.e_intra;
    out.pairs_in = cnt;
    return out;
}

// ---------------------------------------------------------------- pose slots
__device__ __forceinline__ void slot_copy(const Lds& S, int dst, int src, int len)
{
    const int l = lane_id();
    if (l < len) S.pose[dst * kSlot + l] = S.pose[src * kSlot + l];
    wave_sync();
}

// x (+) lam d : t + lam d_t, exp(lam d_theta) q, psi + lam d_psi.  d is the
// lane-distributed tangent vector.
__device__ __forceinline__ void retract(const Lds& S, int dst, int src, float d, float lam, int nt)
{
    const int l = lane_id();
    const float* x = S.pose + src * kSlot;
    float* o = S.pose + dst * kSlot;
    const int np = 7 + nt;
    // one LDS read: lane k holds pose entry k; the quaternion comes from
    // lanes 3..6 by readlane (dst and src are distinct slots)
    const float xv = l < np ? x[l] : 0.f;
    const float th0 = lane_f(d, 3) * lam, th1 = lane_f(d, 4) * lam, th2 = lane_f(d, 5) * lam;
    float dq[4], q[4] = {lane_f(xv, 3), lane_f(xv, 4), lane_f(xv, 5), lane_f(xv, 6)}, nq[4];
    rotvec_quat(th0, th1, th2, dq);
    quat_mul(dq, q, nq);
    quat_normalize(nq);
    // pose entries 0..2 move by tangent lanes 0..2, entry k >= 7 (a torsion)
    // by tangent lane k - 1, brought over by a whole-wave shift (DPP wave_shr:1)
    const float dprev = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(d), 0x138, 0xF, 0xF, false));
    float v = xv + lam * (l < 3 ? d : dprev);
    v = l == 6 ? nq[3] : v;
    v = l == 5 ? nq[2] : v;
    v = l == 4 ? nq[1] : v;
    v = l == 3 ? nq[0] : v;
    if (l < np) o[l] = v;
    wave_sync();
}

// ---------------------------------------------------------------- RILC-BFGS
constexpr int kMaxM = 8;     // the most history pairs a search may keep (bfgs_m)
constexpr int kShortM = 5;   // the dock kernel is also built for at most this many (the default m): the history
                             // lives in registers, and room for 8 pairs cost the shift and copies of 3 more

struct BfgsOut {
    float f;
    float g;          // this lane's tangent gradient component at the result
    int evals;
    int grads;        // evaluations that computed the gradient
    int bounded;      // evaluations decided by the intra lower bound (no pair loop)
    int64_t pairs;    // this lane's share of the intra pairs inside the cutoff
    bool skipped;     // the consistency check ended the run after its first evaluation
    bool outside0;    // the start pose has an atom outside the box
};

// The neighbour of a mutated pose for the first-order consistency check:
// the current pose (LDS slot SLOT_CUR), its energy and this lane's tangent
// gradient component, and the tangent coordinates [p_lo, p_hi) the
// mutation moved.
struct CheckIn {
    float f, g;
    int p_lo, p_hi;
};

__device__ __forceinline__ float fsgn(float v) { return (float)((v > 0.f) - (v < 0.f)); }

// Eqs. qvina_eq_4 and qvina_eq_5 for the pose in `x` (energy fx, this
// lane's gradient gx) against its neighbour: true (optimise) when in some
// tested coordinate the derivative changes sign between the two poses or
// disagrees with the secant slope.  Tangent differences: translation, the
// rotation vector of q_x conj(q_cur) (only its sign is used), torsions
// wrapped to (-pi, pi].
__device__ __forceinline__ bool consistency_passes(const Lds& S, const float* x, float fx, float gx, const CheckIn& ck)
{
    const int l = lane_id();
    const float* y = S.pose + SLOT_CUR * kSlot;
    float dl = 0.f;
    if (l < 3) {
        dl = x[l] - y[l];
    } else if (l < 6) {
        const float qx[4] = {x[3], x[4], x[5], x[6]};
        const float cy[4] = {y[3], -y[4], -y[5], -y[6]};
        float qd[4];
        quat_mul(qx, cy, qd);
        const float v = l == 3 ? qd[1] : (l == 4 ? qd[2] : qd[3]);
        dl = qd[0] < 0.f ? -v : v;
    } else if (l + 1 < kSlot) {
        const float kPi = 3.14159265358979f, k2Pi = 6.28318530717959f;
        float d = x[l + 1] - y[l + 1];
        d -= k2Pi * floorf((d + kPi) * (1.f / k2Pi));
        dl = d == -kPi ? kPi : d;
    }
    const bool in = l >= ck.p_lo && l < ck.p_hi;
    const float sx = fsgn(gx);
    const bool hold = sx * fsgn(ck.g) <= 0.f || sx * fsgn(fx - ck.f) * fsgn(dl) <= 0.f;
    return __ballot(in && hold) != 0;
}

// Minimises from the pose in SLOT_X; the result is left in SLOT_X.  Written
// as one loop around a single evaluation (the first at x0, then one per
// line-search trial) so the kernel carries one copy of the evaluation code.
template <int A, bool SL, int MM = kMaxM>
__device__ BfgsOut bfgs(const Topo<A, SL>& T, const BoxView& B, const Lds& S, const SearchParams& P, int max_iter,
                        bool check = false, CheckIn ck = CheckIn{0.f, 0.f, 0, 0})
{
    static_assert(MM >= 1 && MM <= kMaxM, "history capacity");
    const int l = lane_id();
    const int nd = 6 + T.nt;
    const bool act = l < nd;
    BfgsOut out;
    out.evals = 0;
    out.grads = 0;
    out.bounded = 0;
    out.pairs = 0;
    out.skipped = false;
    out.outside0 = false;
    float Sh[MM], Yh[MM], rh[MM];
#pragma unroll
    for (int h = 0; h < MM; ++h) { Sh[h] = 0.f; Yh[h] = 0.f; rh[h] = 0.f; }
    int hn = 0, it = 0, tr = 0;
    const int m = P.m;
    float f = 0.f, g = 0.f, d = 0.f, gd = 0.f, gn = 0.f;
    float lo = 0.f, lam = 1.f, beta = 0.f, fa = 0.f, ga = 0.f;
    float sy_new = 0.f, yy_new = 1.f;   // s.y and y.y of the newest stored pair (the H0 scale)
    bool beta_inf = true, initial = true;
    while (true) {
        // a trial above the sufficient-decrease bound needs no gradient.  The
        // intra bound decides an iteration's first trial (the full step) less
        // often than the later ones, and with one atom per lane trying it costs
        // the corner loads their cover by the pair loop: that form tries it
        // once a trial of the iteration has failed, and while no history pair
        // is stored, when the full step is the unscaled gradient step
        const float armijo = initial ? __builtin_inff() : f + P.rho * lam * gd;
        const Eval ev = evaluate(T, B, S, S.pose + (initial ? SLOT_X : SLOT_XT) * kSlot, armijo,
                                 !(P.flags & kDockNoIntraBound) && (A > 1 || tr > 0 || hn == 0));
        ++out.evals;
        out.grads += ev.e > armijo ? 0 : 1;
        out.bounded += ev.bounded ? 1 : 0;
        out.pairs += ev.pairs_in;
        const float ft = ev.e, gt = act ? ev.g : 0.f;
        bool begin = false;
        if (initial) {
            f = ft; g = gt; initial = false; begin = true;
            out.outside0 = ev.outside;
            if (check && !consistency_passes(S, S.pose + SLOT_X * kSlot, ft, gt, ck)) {
                out.skipped = true;
                break;
            }
        } else {
            // Lewis-Overton trial at step lam (Eqs. qvina_eq_7 and qvina_eq_8)
            bool accepted = false;
            if (ft > armijo) {
                beta = lam; beta_inf = false;
            } else if (wsum_n(gt * d, nd) < P.sigma * gd) {
                lo = lam;
                slot_copy(S, SLOT_XA, SLOT_XT, 7 + T.nt);
                fa = ft; ga = gt;
            } else {
                accepted = true;
            }
            float lam_ok = lam, fn = ft, gnw = gt;
            if (!accepted) {
                ++tr;
                if (tr < P.ls_max) {
                    lam = beta_inf ? 2.f * lam : 0.5f * (lo + beta);
                    retract(S, SLOT_XT, SLOT_X, d, lam, T.nt);
                    continue;
                }
                if (!(lo > 0.f)) break;
                lam_ok = lo;
                slot_copy(S, SLOT_XT, SLOT_XA, 7 + T.nt);
                fn = fa; gnw = ga;
            }
            // s = lam d, y = g+ - g; cautious update (Eqs. qvina_eq_10, qvina_eq_11)
            const float sv = lam_ok * d, yv = gnw - g;
            const float ys = wsum_n(yv * sv, nd), ss = wsum_n(sv * sv, nd), yy = wsum_n(yv * yv, nd);
            if (ys * __builtin_amdgcn_rcpf(ss) > P.eps_c * gn) {
                sy_new = ys;
                yy_new = yy;
                if (hn == m) {
#pragma unroll
                    for (int h = 0; h < MM - 1; ++h) { Sh[h] = Sh[h + 1]; Yh[h] = Yh[h + 1]; rh[h] = rh[h + 1]; }
                    --hn;
                }
#pragma unroll
                for (int h = 0; h < MM; ++h)
                    if (h == hn) { Sh[h] = sv; Yh[h] = yv; rh[h] = __builtin_amdgcn_rcpf(ys); }
                ++hn;
            }
            slot_copy(S, SLOT_X, SLOT_XT, 7 + T.nt);   // Eq. qvina_eq_9
            f = fn;
            g = gnw;
            ++it;
            begin = true;
        }
        if (begin) {
            if (it >= max_iter) break;
            gn = __builtin_amdgcn_sqrtf(wsum_n(g * g, nd));
            if (gn <= P.eps_g) break;                 // Eq. qvina_eq_12
            // two-loop recursion: d = -H g (d = -g with no pairs, Eq. qvina_eq_6)
            float q = g, al[MM];
#pragma unroll
            for (int h = MM - 1; h >= 0; --h) {
                al[h] = 0.f;
                if (h < hn) {
                    al[h] = rh[h] * wsum_n(Sh[h] * q, nd);
                    q -= al[h] * Yh[h];
                }
            }
            if (hn > 0) q *= sy_new * __builtin_amdgcn_rcpf(yy_new);
#pragma unroll
            for (int h = 0; h < MM; ++h) {
                if (h < hn) {
                    const float bb = rh[h] * wsum_n(Yh[h] * q, nd);
                    q += Sh[h] * (al[h] - bb);
                }
            }
            d = -q;
            gd = wsum_n(g * d, nd);
            if (!(gd < 0.f)) break;                   // not a descent direction
            lo = 0.f; lam = 1.f; beta = 0.f; beta_inf = true; tr = 0;
            retract(S, SLOT_XT, SLOT_X, d, lam, T.nt);
        }
    }
    out.f = f;
    out.g = g;
    return out;
}

// ---------------------------------------------------------------- Monte Carlo
struct ChainOut {
    float best_e;
    int64_t evals, grads, bounded, pairs;   // pairs: this lane's share
    int status;                    // PV_JOB_BUDGET | PV_JOB_OUTSIDE bits
};

constexpr int kStatusBudget = 2, kStatusOutside = 4;   // the PV_JOB_* bits of the ABI

template <int A, bool SL>
__device__ void init_pose(const Topo<A, SL>& T, const BoxView& B, const Lds& S, int slot, uint64_t seed, int job,
                          int chain)
{
    const int l = lane_id();
    // lane l draws uniform l (block l/4, word l%4) of step 0
    const float u = u01(philox_word(seed, job, chain, 0, (uint64_t)(l >> 2), l & 3));
    const float u3 = lane_f(u, 3), u4 = lane_f(u, 4), u5 = lane_f(u, 5);
    const float s1 = sqrtf(1.f - u3), s2 = sqrtf(u3);
    float sa, ca, sb, cb;
    sincosf(2.f * kPi * u4, &sa, &ca);
    sincosf(2.f * kPi * u5, &sb, &cb);
    float* o = S.pose + slot * kSlot;
    if (l == 0) o[0] = B.ox + u * B.ex;
    if (l == 1) o[1] = B.oy + u * B.ey;
    if (l == 2) o[2] = B.oz + u * B.ez;
    if (l == 3) o[3] = s2 * cb;
    if (l == 4) o[4] = s1 * sa;
    if (l == 5) o[5] = s1 * ca;
    if (l == 6) o[6] = s2 * sb;
    if (l >= 6 && l < 6 + T.nt) o[l + 1] = -kPi + 2.f * kPi * u;
    wave_sync();
}

// Mutation of one POT entity (Eq. qvina_eq_2) from the 8 words w of the step.
template <int A, bool SL>
__device__ void mutate(const Topo<A, SL>& T, const Lds& S, int slot, const SearchParams& P, const uint64_t w[8])
{
    const int l = lane_id();
    float* x = S.pose + slot * kSlot;
    const uint64_t n_ent = (uint64_t)(2 + T.nt);
    const int ent = (int)(((w[0] >> 32) * n_ent) >> 32);
    const float u1 = u01(w[1]), u2 = u01(w[2]), u3 = u01(w[3]), u4 = u01(w[4]);
    const float ur = u01(w[5]), ua = u01(w[6]);
    const float r12 = sqrtf(-2.f * logf(1.f - u1)), r34 = sqrtf(-2.f * logf(1.f - u3));
    float s2, c2, s4, c4;
    sincosf(2.f * kPi * u2, &s2, &c2);
    sincosf(2.f * kPi * u4, &s4, &c4);
    const float vx = r12 * c2, vy = r12 * s2, vz = r34 * c4;
    const float vn2 = vx * vx + vy * vy + vz * vz;
    float dx = 0.f, dy = 0.f, dz = 1.f;
    if (vn2 > 0.f) { const float inv = 1.f / sqrtf(vn2); dx = vx * inv; dy = vy * inv; dz = vz * inv; }
    const float rad = cbrtf(ur);
    wave_sync();
    if (ent == 0) {
        const float a = P.pos_amp * rad;
        if (l == 0) x[0] += a * dx;
        if (l == 1) x[1] += a * dy;
        if (l == 2) x[2] += a * dz;
    } else if (ent == 1) {
        const float amp = P.rot_amp * T.rot_scale * rad;
        float dq[4], q[4] = {x[3], x[4], x[5], x[6]}, nq[4];
        rotvec_quat(amp * dx, amp * dy, amp * dz, dq);
        quat_mul(dq, q, nq);
        quat_normalize(nq);
        wave_sync();
        if (l == 3) x[3] = nq[0];
        if (l == 4) x[4] = nq[1];
        if (l == 5) x[5] = nq[2];
        if (l == 6) x[6] = nq[3];
    } else {
        if (l == 7 + (ent - 2)) x[l] = -kPi + 2.f * kPi * ua;
    }
    wave_sync();
}

// Wave priority from the chain's predicted remaining work: its evaluations
// per step so far times the steps left, per step of the whole run.  Waves
// that share a SIMD (or a CU's LDS and memory pipes) then serve the chain
// with the most work left first, which shortens a launch that ends with its
// longest chain.  Arbitration only: the results do not change.
__device__ __forceinline__ void chain_priority(int64_t evals, int s, int steps)
{
    const float q = (float)evals * (float)(steps - s) / ((float)s * (float)steps);
    if (q >= 24.f) __builtin_amdgcn_s_setprio(3);
    else if (q >= 16.f) __builtin_amdgcn_s_setprio(2);
    else if (q >= 8.f) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

template <int A, bool SL, int MM = kMaxM>
__device__ ChainOut mc_chain(const Topo<A, SL>& T, const BoxView& B, const Lds& S, const SearchParams& P, int job,
                             int chain)
{
    const int l = lane_id();
    ChainOut out;
    out.evals = 0;
    out.grads = 0;
    out.bounded = 0;
    out.pairs = 0;
    out.status = 0;
    init_pose(T, B, S, SLOT_X, P.seed, job, chain);
    float e_cur = 0.f, e_best = 0.f, um = 0.f;
    CheckIn ck;            // the current pose as the consistency check's neighbour
    ck.g = 0.f;
    ck.p_lo = ck.p_hi = 0;
    // 0 initial pose, 1 step optimisation, 2 refinement, 3 the closing
    // look at the best pose (one uncounted evaluation: is it inside the box?)
    int s = 0, mode = 0;
    while (true) {
        const int iters = mode == 0 || mode == 3 ? 0 : (mode == 1 ? P.max_iter : P.refine_max_iter);
        ck.f = e_cur;
        const BfgsOut bo = bfgs<A, SL, MM>(T, B, S, P, iters, mode == 1 && P.consistency, ck);
        if (mode == 3) {
            if (bo.outside0) out.status |= kStatusOutside;
            break;
        }
        out.evals += bo.evals;
        out.grads += bo.grads;
        out.bounded += bo.bounded;
        out.pairs += bo.pairs;
        bool next = true;
        if (mode == 0) {
            e_cur = e_best = bo.f;
            ck.g = bo.g;
            slot_copy(S, SLOT_CUR, SLOT_X, 7 + T.nt);
            slot_copy(S, SLOT_BEST, SLOT_X, 7 + T.nt);
        } else if (mode == 1) {
            if (!bo.skipped) {
                const float e_o = bo.f;
                if (e_o < e_cur || um < __expf((e_cur - e_o) / P.temperature)) {   // Eq. qvina_eq_13
                    slot_copy(S, SLOT_CUR, SLOT_X, 7 + T.nt);
                    e_cur = e_o;
                    ck.g = bo.g;
                }
                if (e_o < e_best) { mode = 2; next = false; }
            }
        } else {
            slot_copy(S, SLOT_BEST, SLOT_X, 7 + T.nt);
            slot_copy(S, SLOT_CUR, SLOT_X, 7 + T.nt);
            e_best = bo.f;
            e_cur = bo.f;
            ck.g = bo.g;
        }
        if (!next) continue;
        const bool spent = P.max_evals > 0 && out.evals >= P.max_evals;
        if (spent) out.status |= kStatusBudget;
        if (s >= P.steps || spent) {
            slot_copy(S, SLOT_X, SLOT_BEST, 7 + T.nt);
            mode = 3;
            continue;
        }
        // the 8 draws of step s + 1: lanes 0-3 compute block 0, lanes 4-7 block 1
        const uint64_t mine = philox_word(P.seed, job, chain, (uint64_t)s + 1, (uint64_t)((l >> 2) & 1), l & 3);
        uint64_t w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t lo = (uint32_t)lane_i((int)(uint32_t)mine, k);
            const uint32_t hi = (uint32_t)lane_i((int)(uint32_t)(mine >> 32), k);
            w[k] = ((uint64_t)hi << 32) | lo;
        }
        um = u01(w[7]);
        // tangent coordinates the mutation moves (its entity draw, as in mutate)
        const int ent = (int)(((w[0] >> 32) * (uint64_t)(2 + T.nt)) >> 32);
        ck.p_lo = ent == 0 ? 0 : (ent == 1 ? 3 : 4 + ent);
        ck.p_hi = ent <= 1 ? ck.p_lo + 3 : ck.p_lo + 1;
        slot_copy(S, SLOT_X, SLOT_CUR, 7 + T.nt);
        mutate(T, S, SLOT_X, P, w);
        ++s;
        mode = 1;
        chain_priority(out.evals, s, P.steps);
    }
    __builtin_amdgcn_s_setprio(0);
    out.best_e = e_best;
    return out;
}

// ---------------------------------------------------------------- kernels

// Two waves per SIMD for the slot form and the two-atom form: without the
// hint they take AGPRs above 256 VGPRs and fall to one wave (with it the slot
// form holds 247 VGPRs, the two-atom form 256 with 28 spilled).  The one-atom
// gather form fits two waves by itself and is faster without the hint.
template <int A, bool SL, int MM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SL || A > 1 ? 2 : 1))) void dock_kernel(DockArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const Lds S = carve(smem, a.l.max_atoms, a.l.max_pairs, a.l.max_ell, kernel_needs(kKindDock, A, SL));
    const int l = lane_id();
    Topo<A, SL> T;
    T.lig = -1;
    const int chains = a.sp.chains;
    int64_t item = a.persistent ? -1 : (int64_t)blockIdx.x;
    while (true) {
        if (a.persistent) {
            uint32_t v = 0;
            if (l == 0) v = atomicAdd(a.queue, 1u);
            item = (int64_t)(uint32_t)lane_i((int)v, 0);
        }
        if (item >= a.n_items) break;
        const int gj = (int)(item / chains);
        const int job = a.job_map ? a.job_map[gj] : a.job_begin + gj;
        const int chain = (int)(item % chains);
        const int2 jb = a.jobs[job];
        if (jb.x != T.lig) stage_ligand(T, a.l, jb.x, S);
        const BoxView B = box_view(a.g, jb.y);
        uint64_t t0 = 0;
        if (a.sp.flags & 1u) t0 = wall_clock64();
        ChainOut co = mc_chain<A, SL, MM>(T, B, S, a.sp, job, chain);
        const int64_t pairs = wsum_i64(co.pairs);
        const int64_t ci = (int64_t)job * chains + chain;
        if (a.chain_best_dof && l < a.dof_stride)
            a.chain_best_dof[ci * a.dof_stride + l] = l < 7 + T.nt ? S.pose[SLOT_BEST * kSlot + l] : 0.f;
        if (l == 0) {
            if (a.chain_best_e) a.chain_best_e[ci] = co.best_e;
            if (a.chain_evals) a.chain_evals[ci] = co.evals;
            if (a.chain_pairs) a.chain_pairs[ci] = pairs;
            if (a.chain_grads) a.chain_grads[ci] = co.grads;
            if (a.chain_bounded) a.chain_bounded[ci] = co.bounded;
            a.chain_status[ci] = co.status;
            if (a.sp.flags & 1u) {
                const uint64_t t1 = wall_clock64();
                atomicMin((unsigned long long*)&a.job_t_start[job], (unsigned long long)t0);
                atomicMax((unsigned long long*)&a.job_t_end[job], (unsigned long long)t1);
            }
        }
        wave_sync();
        if (!a.persistent) break;
    }
}

__global__ void reset_queue_kernel(uint32_t* q) { if (threadIdx.x == 0) *q = 0u; }

// Measurement aid, the VALU FP32 issue rate: every thread runs 16 independent
// multiply-add chains for `iters` rounds with no memory traffic and stores
// their sum once, so the launch is bound by FMA issue alone.
__global__ __launch_bounds__(256) void fma_peak_kernel(float* out, int iters)
{
    const int gid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const float a = 0.999999f, b = 1e-7f * (float)(threadIdx.x & 7u);
    float x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = (float)(gid + k) * 1e-6f;
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = fmaf(x[k], a, b);
    }
    float sum = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += x[k];
    out[gid] = sum;
}

__global__ void reset_times_kernel(uint64_t* t0, uint64_t* t1, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { t0[i] = ~0ull; t1[i] = 0ull; }
}

// Per job: the best chain (lowest energy, ties to the lower chain, a number
// before NaN), the evaluation total and the status bits: not finite, some
// chain stopped at its budget, the best chain's pose outside the box.
__global__ void job_reduce_kernel(const float* cbe, const int64_t* cev, const int32_t* cst, int n_jobs, int chains,
                                  float* jbe, int32_t* jbc, int64_t* jev, int32_t* jst)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_jobs) return;
    int bc = 0;
    float be = cbe[(int64_t)j * chains];
    int64_t ev = cev ? cev[(int64_t)j * chains] : 0;
    int budget = cst[(int64_t)j * chains] & kStatusBudget;
    for (int c = 1; c < chains; ++c) {
        const float e = cbe[(int64_t)j * chains + c];
        if (e < be || (be != be && e == e)) { be = e; bc = c; }
        if (cev) ev += cev[(int64_t)j * chains + c];
        budget |= cst[(int64_t)j * chains + c] & kStatusBudget;
    }
    if (jbe) jbe[j] = be;
    if (jbc) jbc[j] = bc;
    if (jev) jev[j] = ev;
    if (jst) jst[j] = (isfinite(be) ? 0 : 1) | budget | (cst[(int64_t)j * chains + bc] & kStatusOutside);
}

// The one-atom gather form fits three waves per SIMD in 168 VGPRs (4 of them
// spilled to scratch; three waves measured 10% faster than two); the other
// forms need more.
template <int A, bool SL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(A == 1 && !SL ? 3 : 1))) void score_kernel(ScoreArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const Lds S = carve(smem, a.l.max_atoms, a.l.max_pairs, a.l.max_ell, kernel_needs(kKindScore, A, SL));
    const int l = lane_id();
    Topo<A, SL> T;
    T.lig = -1;
    const float nanv = __int_as_float(0x7fc00000);
    // a contiguous run of poses per workgroup (runs of one ligand stage it
    // once), the runs' lengths differing by at most one so no wave idles
    const int p_begin = (int)(((int64_t)blockIdx.x * a.n_poses) / (int64_t)gridDim.x);
    const int p_end = (int)(((int64_t)(blockIdx.x + 1) * a.n_poses) / (int64_t)gridDim.x);
    // the next pose's indices and pose vector are loaded while this one is
    // evaluated (lane l holds pose entry l)
    const bool dof_in = !a.from_xyz;
    int n_lig = 0, n_box = 0;
    float n_dof = 0.f;
    if (p_begin < p_end) {
        n_lig = a.lig_of_pose[p_begin];
        n_box = a.box_of_pose[p_begin];
        if (dof_in && l < a.dof_stride) n_dof = a.dof[(int64_t)p_begin * a.dof_stride + l];
    }
    for (int pose = p_begin; pose < p_end; ++pose) {
        const int lig = n_lig, box = n_box;
        const float dof_l = n_dof;
        if (pose + 1 < p_end) {
            n_lig = a.lig_of_pose[pose + 1];
            n_box = a.box_of_pose[pose + 1];
            if (dof_in && l < a.dof_stride) n_dof = a.dof[(int64_t)(pose + 1) * a.dof_stride + l];
        }
        if (lig < 0 || lig >= a.l.n_lig || box < 0 || box >= a.g.n_boxes) {
            if (l == 0 && a.energy) a.energy[pose] = nanv;
            if (l < 2 && a.e_parts) a.e_parts[2 * (int64_t)pose + l] = nanv;
            if (a.grad_dof && l < a.dof_stride) a.grad_dof[(int64_t)pose * a.dof_stride + l] = nanv;
            for (int k = l; k < 3 * a.xyz_stride; k += kWave) {
                if (a.xyz_out && !a.from_xyz) a.xyz_out[(int64_t)pose * a.xyz_stride * 3 + k] = nanv;
                if (a.grad_xyz) a.grad_xyz[(int64_t)pose * a.xyz_stride * 3 + k] = nanv;
            }
            continue;
        }
        if (lig != T.lig) stage_ligand(T, a.l, lig, S);
        const BoxView B = box_view(a.g, box);
        const float scale = a.grad_energy ? a.grad_energy[pose] : 1.f;
        const int16_t* perm = a.l.perm + a.l.ligs[lig].atom_base;
        Eval ev;
        if (!a.from_xyz) {
            if (l < 7 + T.nt) S.pose[SLOT_X * kSlot + l] = dof_l;
            wave_sync();
            ev = evaluate(T, B, S, S.pose + SLOT_X * kSlot);
        } else {
            for (int i = l; i < T.n; i += kWave) {
                const float* src = a.dof + ((int64_t)pose * a.xyz_stride + perm[i]) * 3;
                S.pos[i] = make_float4(src[0], src[1], src[2], 0.f);
            }
            wave_sync();
            ev = evaluate_xyz(T, B, S);
        }
        if (l == 0 && a.energy) a.energy[pose] = ev.e;
        if (a.e_parts && l < 2) a.e_parts[2 * (int64_t)pose + l] = l == 0 ? ev.e_inter : ev.e_intra;
        if (a.grad_dof && !a.from_xyz) {
            // dE/dt, dE/d(raw q) = 2 ((0, torque) (x) q)/|p|, dE/dpsi
            const float* x = S.pose + SLOT_X * kSlot;
            const float tq0 = lane_f(ev.g, 3), tq1 = lane_f(ev.g, 4), tq2 = lane_f(ev.g, 5);
            const float dpsi = __shfl(ev.g, l - 1 < 0 ? 0 : (l - 1 > 63 ? 63 : l - 1));
            float p[4] = {x[3], x[4], x[5], x[6]};
            const float pn = sqrtf(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
            float qh[4] = {p[0] / pn, p[1] / pn, p[2] / pn, p[3] / pn};
            float t4[4] = {0.f, tq0, tq1, tq2}, gq[4];
            quat_mul(t4, qh, gq);
            float v = 0.f;
            if (l < 3) v = ev.g;
            if (l == 3) v = 2.f * gq[0] / pn;
            if (l == 4) v = 2.f * gq[1] / pn;
            if (l == 5) v = 2.f * gq[2] / pn;
            if (l == 6) v = 2.f * gq[3] / pn;
            if (l >= 7 && l < 7 + T.nt) v = dpsi;
            if (l < a.dof_stride) a.grad_dof[(int64_t)pose * a.dof_stride + l] = l < 7 + T.nt ? v * scale : 0.f;
        }
        if (a.xyz_out || a.grad_xyz) {
            // rows past the ligand's atoms (a batch of mixed sizes) are zero
            for (int k = 3 * T.n + l; k < 3 * a.xyz_stride; k += kWave) {
                if (a.xyz_out && !a.from_xyz) a.xyz_out[(int64_t)pose * a.xyz_stride * 3 + k] = 0.f;
                if (a.grad_xyz) a.grad_xyz[(int64_t)pose * a.xyz_stride * 3 + k] = 0.f;
            }
            for (int i = l; i < T.n; i += kWave) {
                const int64_t o = ((int64_t)pose * a.xyz_stride + perm[i]) * 3;
                if (a.xyz_out) {
                    const float4 p = S.pos[i];
                    a.xyz_out[o] = p.x; a.xyz_out[o + 1] = p.y; a.xyz_out[o + 2] = p.z;
                }
                if (a.grad_xyz) {
                    const float4 f = S.frc[i];
                    a.grad_xyz[o] = f.x * scale; a.grad_xyz[o + 1] = f.y * scale; a.grad_xyz[o + 2] = f.z * scale;
                }
            }
        }
        wave_sync();
    }
}

template <int A, bool SL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SL || A > 1 ? 2 : 1))) void local_opt_kernel(OptArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const Lds S = carve(smem, a.l.max_atoms, a.l.max_pairs, a.l.max_ell, kernel_needs(kKindOpt, A, SL));
    const int l = lane_id();
    Topo<A, SL> T;
    T.lig = -1;
    for (int pose = blockIdx.x; pose < a.n_poses; pose += gridDim.x) {
        const int lig = a.lig_of_pose[pose], box = a.box_of_pose[pose];
        if (lig < 0 || lig >= a.l.n_lig || box < 0 || box >= a.g.n_boxes) {
            if (l == 0 && a.energy) a.energy[pose] = __int_as_float(0x7fc00000);
            continue;
        }
        if (lig != T.lig) stage_ligand(T, a.l, lig, S);
        const BoxView B = box_view(a.g, box);
        float v = l < 7 + T.nt ? a.dof_in[(int64_t)pose * a.dof_stride + l] : 0.f;
        // normalise the quaternion once so the run starts from a unit q
        float q0 = lane_f(v, 3), q1 = lane_f(v, 4), q2 = lane_f(v, 5), q3 = lane_f(v, 6);
        const float qn = rsqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
        if (l >= 3 && l < 7) v *= qn;
        if (l < 7 + T.nt) S.pose[SLOT_X * kSlot + l] = v;
        wave_sync();
        BfgsOut bo = bfgs(T, B, S, a.sp, a.sp.max_iter);
        if (l < a.dof_stride) a.dof_out[(int64_t)pose * a.dof_stride + l] = l < 7 + T.nt ? S.pose[SLOT_X * kSlot + l] : 0.f;
        if (l == 0) {
            if (a.energy) a.energy[pose] = bo.f;
            if (a.n_evals) a.n_evals[pose] = bo.evals;
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------- output stage
// Atom positions of the pose in `pose` (an LDS slot) into S.pos.
template <int A, bool SL>
__device__ void pose_positions(const Topo<A, SL>& T, const Lds& S, const float* pose)
{
    const int l = lane_id();
    float R[9], b[3];
    frames(T, S, pose, R, b);
    if (l < T.nf) {
        float* fr = S.frame + 12 * l;
#pragma unroll
        for (int k = 0; k < 9; ++k) fr[k] = R[k];
        fr[9] = b[0]; fr[10] = b[1]; fr[11] = b[2];
    }
    wave_sync();
#pragma unroll
    for (int a = 0; a < A; ++a) {
        const int i = l * A + a;
        if (i < T.n) S.pos[i] = atom_position(T.ref[a], S);
    }
    wave_sync();
}

// Order of the output stage: a before b for a smaller energy, any number
// before NaN, then the lower index.
__device__ __forceinline__ bool precedes(float ea, int ia, float eb, int ib)
{
    const bool na = ea != ea, nb = eb != eb;
    if (na != nb) return nb;
    if (!na && ea != eb) return ea < eb;
    return ia < ib;
}

// Sum over atoms of |S.pos - other|^2 (identical in every lane).
template <int A, bool SL>
__device__ __forceinline__ float sq_dev(const Topo<A, SL>& T, const Lds& S, const float4* other)
{
    const int l = lane_id();
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < A; ++a) {
        const int i = l * A + a;
        if (i < T.n) {
            const float4 p = S.pos[i], q = other[i];
            const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
            s += dx * dx + dy * dy + dz * dz;
        }
    }
    return wsum(s);
}

// One wave per job (Methods, end of "Accelerated Docking with QuickVina
// 2-GPU 2.1"; last steps of Supplementary Algorithm 2): the chains' best
// poses in ascending energy; greedy r.m.s.d. clustering keeps a pose unless
// it lies within rmsd_cut of a kept one, up to `modes`; each kept pose is
// refined by BFGS and rescored (E, and the affinity e_inter / (1 + w T));
// the refined poses are sorted again, filtered by r.m.s.d. the same way and
// written out.  r.m.s.d. < cut is tested as sum |dx|^2 < cut^2 N.
template <int A>
__global__ __launch_bounds__(64) void output_kernel(OutputArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const Lds S = carve(smem, a.l.max_atoms, a.l.max_pairs, a.l.max_ell, kernel_needs(kKindOutput, A, false));
    char* ext = smem + lds_bytes(a.l.max_atoms, a.l.max_pairs, a.l.max_ell, kernel_needs(kKindOutput, A, false));
    const int ma = S.ma, M = a.modes, C = a.chains;
    int* order = (int*)ext;     ext += round_up(C, 4) * 4;
    float4* rep = (float4*)ext; ext += M * ma * 16;
    float* rdof = (float*)ext;  ext += M * kSlot * 4;
    float* re = (float*)ext;    ext += round_up(M, 4) * 4;
    float* ra = (float*)ext;    ext += round_up(M, 4) * 4;
    int* kc = (int*)ext;        ext += round_up(M, 4) * 4;
    int* fo = (int*)ext;        ext += round_up(M, 4) * 4;
    int* so = (int*)ext;
    const int l = lane_id();
    const int job = blockIdx.x;
    Topo<A, false> T;
    T.lig = -1;
    const int2 jb = a.jobs[job];
    stage_ligand(T, a.l, jb.x, S);
    const BoxView B = box_view(a.g, jb.y);
    const float* ce = a.chain_e + (int64_t)job * C;
    const float cut2n = a.rmsd_cut * a.rmsd_cut * (float)T.n;
    float* x = S.pose + SLOT_X * kSlot;
    // 1. chains in ascending energy (rank of each chain by counting)
    for (int c = l; c < C; c += kWave) {
        const float ec = ce[c];
        int rank = 0;
        for (int c2 = 0; c2 < C; ++c2) rank += precedes(ce[c2], c2, ec, c) ? 1 : 0;
        order[rank] = c;
    }
    wave_sync();
    // 2. greedy clustering in that order
    int nk = 0;
    for (int r = 0; r < C && nk < M; ++r) {
        const int c = order[r];
        const float* src = a.chain_dof + ((int64_t)job * C + c) * a.in_stride;
        if (l < 7 + T.nt) x[l] = src[l];
        wave_sync();
        pose_positions(T, S, x);
        bool keep = true;
        for (int q = 0; q < nk && keep; ++q) keep = !(sq_dev(T, S, rep + q * ma) < cut2n);
        if (keep) {
#pragma unroll
            for (int aa = 0; aa < A; ++aa) {
                const int i = l * A + aa;
                if (i < T.n) rep[nk * ma + i] = S.pos[i];
            }
            if (l == 0) kc[nk] = c;
            ++nk;
        }
        wave_sync();
    }
    // 3. refine and rescore every kept pose
    for (int q = 0; q < nk; ++q) {
        const float* src = a.chain_dof + ((int64_t)job * C + kc[q]) * a.in_stride;
        if (l < 7 + T.nt) x[l] = src[l];
        wave_sync();
        if (a.refine_max_iter > 0) bfgs(T, B, S, a.sp, a.refine_max_iter);
        // a unit quaternion, then the rescoring evaluation
        float v = l < 7 + T.nt ? x[l] : 0.f;
        const float q0 = lane_f(v, 3), q1 = lane_f(v, 4), q2 = lane_f(v, 5), q3 = lane_f(v, 6);
        const float qn = 1.f / sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
        if (l >= 3 && l < 7) v *= qn;
        wave_sync();
        if (l < 7 + T.nt) x[l] = v;
        wave_sync();
        const Eval ev = evaluate(T, B, S, x);
#pragma unroll
        for (int aa = 0; aa < A; ++aa) {
            const int i = l * A + aa;
            if (i < T.n) rep[q * ma + i] = S.pos[i];
        }
        if (l < kSlot) rdof[q * kSlot + l] = v;
        if (l == 0) {
            re[q] = ev.e;
            ra[q] = ev.e_inter / (1.f + a.affinity_w * (float)T.nt);
        }
        wave_sync();
    }
    // 4. final sort of the refined poses, r.m.s.d. filter, output
    if (l < nk) {
        int rank = 0;
        for (int q2 = 0; q2 < nk; ++q2) rank += precedes(re[q2], q2, re[l], l) ? 1 : 0;
        fo[rank] = l;
    }
    wave_sync();
    const int64_t o0 = (int64_t)job * M;
    int no = 0;
    for (int r = 0; r < nk; ++r) {
        const int q = fo[r];
        // S.pos <- refined pose q, compared with the poses already written
#pragma unroll
        for (int aa = 0; aa < A; ++aa) {
            const int i = l * A + aa;
            if (i < T.n) S.pos[i] = rep[q * ma + i];
        }
        wave_sync();
        bool keep = true;
        for (int s2 = 0; s2 < no && keep; ++s2) keep = !(sq_dev(T, S, rep + so[s2] * ma) < cut2n);
        if (keep) {
            if (l == 0) {
                so[no] = q;
                a.mode_chain[o0 + no] = kc[q];
                a.mode_e[o0 + no] = re[q];
                if (a.mode_affinity) a.mode_affinity[o0 + no] = ra[q];
            }
            if (a.mode_dof && l < a.out_stride)
                a.mode_dof[(o0 + no) * a.out_stride + l] = l < 7 + T.nt ? rdof[q * kSlot + l] : 0.f;
            ++no;
        }
        wave_sync();
    }
    const float nanv = __int_as_float(0x7fc00000);
    for (int o = no + l; o < M; o += kWave) {
        a.mode_chain[o0 + o] = -1;
        a.mode_e[o0 + o] = nanv;
        if (a.mode_affinity) a.mode_affinity[o0 + o] = nanv;
    }
    if (a.mode_dof)
        for (int o = no; o < M; ++o)
            if (l < a.out_stride) a.mode_dof[(o0 + o) * a.out_stride + l] = 0.f;
    if (l == 0) a.n_modes[job] = no;
}

// ---------------------------------------------------------------- grid maps
// One workgroup per 16x4x4 tile of one box (a wave writes 16-float = 64 B
// rows).  A term enters the sum when r < 8 A, decided in binary32 where that
// is unambiguous and in binary64 near the cutoff.  Receptor atoms near the box are
// streamed in chunks of 256; those within reach of the tile's bounding box
// are compacted into LDS in the atoms' order (a ballot per wave, the waves'
// counts in wave order), so every point sums its terms in the same order on
// every build and the maps are reproducible bit for bit; every lane adds the
// candidates' terms to its point's 8 accumulators (one per ligand type).
constexpr int kGridThreads = kTileX * kTileY * kTileZ;  // 256

// The 8 A cutoff of a map term as r < 8 on binary64 values: the lattice
// point origin + h i, the differences, squares and sum each rounded on its
// own (no contraction), then the correctly rounded square root.  Used for
// the few (point, atom) pairs whose binary32 squared distance lies within
// 0.01 A^2 of 64, where binary32 rounding could decide the other way.
__device__ __noinline__ bool within_cutoff_f64(int i, int j, int k, float ox, float oy, float oz, float h, float4 at)
{
#pragma clang fp contract(off)
    const double gx = (double)ox + (double)h * (double)i;
    const double gy = (double)oy + (double)h * (double)j;
    const double gz = (double)oz + (double)h * (double)k;
    const double dx = gx - (double)at.x, dy = gy - (double)at.y, dz = gz - (double)at.z;
    const double s = dx * dx + dy * dy + dz * dz;
    return __builtin_sqrt(s) < 8.0;
}

__global__ __launch_bounds__(256) void gridmap_kernel(GridBuildArgs a)
{
    __shared__ float4 cand[kGridThreads];
    __shared__ int wave_n[kGridThreads / kWave];
    const int wv = threadIdx.x / kWave;
    // which box and which tile of it
    const int tile = blockIdx.x;
    int box = 0;
    while (box + 1 < a.n_boxes && a.tile_off[box + 1] <= tile) ++box;
    const int nx = a.dims[4 * box], ny = a.dims[4 * box + 1], nz = a.dims[4 * box + 2];
    const float ox = a.geom[8 * box], oy = a.geom[8 * box + 1], oz = a.geom[8 * box + 2], h = a.geom[8 * box + 3];
    const int tx = (nx + kTileX - 1) / kTileX, ty = (ny + kTileY - 1) / kTileY;
    const int t = tile - a.tile_off[box];
    const int bx = t % tx, by = (t / tx) % ty, bz = t / (tx * ty);
    const int li = threadIdx.x % kTileX, lj = (threadIdx.x / kTileX) % kTileY, lk = threadIdx.x / (kTileX * kTileY);
    const int i = bx * kTileX + li, j = by * kTileY + lj, k = bz * kTileZ + lk;
    const bool valid = i < nx && j < ny && k < nz;
    // the lattice point exactly as the cutoff test defines it
    const float gx = fmaf((float)i, h, ox), gy = fmaf((float)j, h, oy), gz = fmaf((float)k, h, oz);
    // tile bounding box (points that exist)
    const float lox = fmaf((float)(bx * kTileX), h, ox), loy = fmaf((float)(by * kTileY), h, oy),
                loz = fmaf((float)(bz * kTileZ), h, oz);
    const float hix = fmaf((float)min(bx * kTileX + kTileX - 1, nx - 1), h, ox);
    const float hiy = fmaf((float)min(by * kTileY + kTileY - 1, ny - 1), h, oy);
    const float hiz = fmaf((float)min(bz * kTileZ + kTileZ - 1, nz - 1), h, oz);
    const float reach2 = 8.01f * 8.01f;
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int abeg = a.atom_off[box], aend = a.atom_off[box + 1];
    // element radii C N O S and the receptor-type table
    const float Rel[4] = {1.9f, 1.8f, 1.7f, 2.0f};
    for (int base = abeg; base < aend; base += kGridThreads) {
        const int ai = base + threadIdx.x;
        bool keep = false;
        float4 at = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ai < aend) {
            at = a.atoms[ai];
            const float ddx = fmaxf(fmaxf(lox - at.x, at.x - hix), 0.f);
            const float ddy = fmaxf(fmaxf(loy - at.y, at.y - hiy), 0.f);
            const float ddz = fmaxf(fmaxf(loz - at.z, at.z - hiz), 0.f);
            keep = ddx * ddx + ddy * ddy + ddz * ddz < reach2;
        }
        // the barrier that ends each chunk has let every reader of the last
        // chunk's wave_n and cand pass, so both may be rewritten here
        const uint64_t m = __ballot(keep);
        if ((threadIdx.x & (kWave - 1)) == 0) wave_n[wv] = __popcll(m);
        __syncthreads();
        int off = 0, nc = 0;
#pragma unroll
        for (int q = 0; q < kGridThreads / kWave; ++q) {
            const int c = wave_n[q];
            off += q < wv ? c : 0;
            nc += c;
        }
        if (keep)
            cand[off + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = at;
        __syncthreads();
        for (int c = 0; c < nc; ++c) {
            const float4 at = cand[c];
            const float dx = gx - at.x, dy = gy - at.y, dz = gz - at.z;
            const float dz2 = dz * dz;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz2));
            if (!(r2 < kCut2 + 0.01f)) continue;
            if (r2 > kCut2 - 0.01f && !within_cutoff_f64(i, j, k, ox, oy, oz, h, at)) continue;
            const float r = __builtin_amdgcn_sqrtf(r2);
            const int rt = __float_as_uint(at.w) & 0xff;
            const float Rr = rt <= 1 ? 1.9f : rt <= 4 ? 1.8f : rt <= 6 ? 1.7f : 2.0f;
            const bool r_hyd = rt == 0, r_don = rt == 3 || rt == 6, r_acc = rt == 4 || rt == 5 || rt == 6;
            float base_e[4], hbv[4];
            float hyd_c = 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float d = r - (Rel[e] + Rr);
                const float g1 = __expf(-4.f * d * d);
                const float dm3 = d - 3.f;
                const float g2 = __expf(-0.25f * dm3 * dm3);
                float v = kW1 * g1 + kW2 * g2;
                if (d < 0.f) v += kW3 * d * d;
                base_e[e] = v;
                hbv[e] = d < -0.7f ? 1.f : (d < 0.f ? -d * (1.f / 0.7f) : 0.f);
                if (e == 0) hyd_c = d < 0.5f ? 1.f : (d < 1.5f ? 1.5f - d : 0.f);
            }
            acc[0] += base_e[0] + (r_hyd ? kW4 * hyd_c : 0.f);           // C_H
            acc[1] += base_e[0];                                         // C_P
            acc[2] += base_e[1];                                         // N_P
            acc[3] += base_e[1] + (r_acc ? kW5 * hbv[1] : 0.f);          // N_D
            acc[4] += base_e[1] + (r_don ? kW5 * hbv[1] : 0.f);          // N_A
            acc[5] += base_e[2] + (r_don ? kW5 * hbv[2] : 0.f);          // O_A
            acc[6] += base_e[2] + ((r_don || r_acc) ? kW5 * hbv[2] : 0.f); // O_DA
            acc[7] += base_e[3];                                         // S_P
        }
        __syncthreads();
    }
    if (valid) {
        const int64_t msz = (int64_t)nx * ny * nz;
        const int64_t idx = ((int64_t)k * ny + j) * nx + i;
        float* out = a.maps + a.map_off[box];
#pragma unroll
        for (int tt = 0; tt < 8; ++tt) out[tt * msz + idx] = acc[tt];
    }
}

// ---------------------------------------------------------------- surface points
// The step before the path (Methods, "Pocket prediction with P2Rank"):
// solvent-accessible surface points of the receptor and their Eq.
// prank_eq_1 features.  Atom records are float4 (x, y, z, type bits) with
// the expanded radius r = X-Score radius + probe computed in binary32.
constexpr int kSasThreads = 256;

__device__ __forceinline__ float sas_radius(int t, float probe)
{
    const float R = t <= 1 ? 1.9f : (t <= 4 ? 1.8f : (t <= 6 ? 1.7f : 2.0f));
    return R + probe;
}

// One thread per candidate c = x_a + r_a u_k (atom-major); the receptor is
// streamed through LDS.  A candidate strictly inside another atom's
// expanded sphere is dropped.  Writes the candidate, its keep flag and the
// block's kept count.
__global__ __launch_bounds__(kSasThreads) void sas_candidates_kernel(const float4* atoms, int n_rec, const float* dirs,
                                                                     int n_dirs, float probe, int64_t n_cand,
                                                                     float4* cand, uint8_t* keep, int32_t* block_count)
{
    __shared__ float4 tile[kSasThreads];
    __shared__ int count;
    const int64_t idx = (int64_t)blockIdx.x * kSasThreads + threadIdx.x;
    const bool valid = idx < n_cand;
    int a = 0;
    float cx = 0.f, cy = 0.f, cz = 0.f;
    if (valid) {
        a = (int)(idx / n_dirs);
        const int k = (int)(idx % n_dirs);
        const float4 xa = atoms[a];
        const float ra = sas_radius(__float_as_uint(xa.w) & 0xff, probe);
        cx = __builtin_fmaf(ra, dirs[3 * k], xa.x);
        cy = __builtin_fmaf(ra, dirs[3 * k + 1], xa.y);
        cz = __builtin_fmaf(ra, dirs[3 * k + 2], xa.z);
    }
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    bool buried = false;
    for (int base = 0; base < n_rec; base += kSasThreads) {
        __syncthreads();
        const int b = base + threadIdx.x;
        if (b < n_rec) {
            const float4 xb = atoms[b];
            const float rb = sas_radius(__float_as_uint(xb.w) & 0xff, probe);
            tile[threadIdx.x] = make_float4(xb.x, xb.y, xb.z, rb * rb);
        }
        __syncthreads();
        const int nb = min(kSasThreads, n_rec - base);
        if (valid && !buried)
            for (int j = 0; j < nb; ++j) {
                const float4 t = tile[j];
                const float dx = cx - t.x, dy = cy - t.y, dz = cz - t.z;
                const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                if (d2 < t.w && base + j != a) { buried = true; break; }
            }
    }
    if (valid) {
        cand[idx] = make_float4(cx, cy, cz, __int_as_float(a));
        keep[idx] = buried ? 0 : 1;
        if (!buried) atomicAdd(&count, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) block_count[blockIdx.x] = count;
}

// Kept candidates to their place: the block's offset plus the number of
// kept candidates before this one in the block (in candidate order).
__global__ __launch_bounds__(kSasThreads) void sas_scatter_kernel(const float4* cand, const uint8_t* keep,
                                                                  const int32_t* block_offset, int64_t n_cand,
                                                                  float4* pts)
{
    __shared__ int pre[kSasThreads];
    const int64_t idx = (int64_t)blockIdx.x * kSasThreads + threadIdx.x;
    const int k = idx < n_cand ? keep[idx] : 0;
    pre[threadIdx.x] = k;
    __syncthreads();
    for (int off = 1; off < kSasThreads; off <<= 1) {   // inclusive scan in the block
        const int v = threadIdx.x >= off ? pre[threadIdx.x - off] : 0;
        __syncthreads();
        pre[threadIdx.x] += v;
        __syncthreads();
    }
    if (k) pts[block_offset[blockIdx.x] + pre[threadIdx.x] - 1] = cand[idx];
}

// Eq. prank_eq_1 per point: channels 0..7 the one-hot XS type, 8..10 the
// hydrophobic, donor and acceptor flags, each summing max(0, 1 - d/6) over
// atoms with d^2 < 36; channel 11 counts the atoms with d^2 < 100 (the
// protrusion).  One thread per point, receptor streamed through LDS.
__global__ __launch_bounds__(kSasThreads) void sas_features_kernel(const float4* atoms, int n_rec, const float4* pts,
                                                                   int n_pts, float* feat)
{
    __shared__ float4 tile[kSasThreads];
    const int p = blockIdx.x * kSasThreads + threadIdx.x;
    const bool valid = p < n_pts;
    const float4 c = valid ? pts[p] : make_float4(0.f, 0.f, 0.f, 0.f);
    float f[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) f[k] = 0.f;
    for (int base = 0; base < n_rec; base += kSasThreads) {
        __syncthreads();
        if (base + threadIdx.x < n_rec) tile[threadIdx.x] = atoms[base + threadIdx.x];
        __syncthreads();
        const int nb = min(kSasThreads, n_rec - base);
        for (int j = 0; j < nb; ++j) {
            const float4 t = tile[j];
            const float dx = c.x - t.x, dy = c.y - t.y, dz = c.z - t.z;
            const float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
            f[11] += d2 < 100.f ? 1.f : 0.f;
            if (d2 < 36.f) {
                const float w = 1.f - __builtin_amdgcn_sqrtf(d2) * (1.f / 6.f);
                const int ty = __float_as_uint(t.w) & 0xff;
#pragma unroll
                for (int k = 0; k < 8; ++k) f[k] += ty == k ? w : 0.f;
                f[8] += ty == 0 ? w : 0.f;
                f[9] += (ty == 3 || ty == 6) ? w : 0.f;
                f[10] += (ty == 4 || ty == 5 || ty == 6) ? w : 0.f;
            }
        }
    }
    if (valid)
#pragma unroll
        for (int k = 0; k < 12; ++k) feat[(int64_t)p * 12 + k] = f[k];
}

// ---------------------------------------------------------------- allocation-free scratch
// The allocation-free dock entry point keeps its scratch (kNoAllocBytes,
// laid out by noalloc_layout) in this array.  Each GPU the library runs on
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel: it takes the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

hipError_t noalloc_scratch(void** out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

// Stable split of the jobs into the two size classes, in chunks of 1024:
// a ballot per wave ranks the members of each class inside the wave, and
// the waves' counts, added in wave order, place them after the earlier
// chunks.  Also zeroes the classes' queue counters.
__global__ __launch_bounds__(1024) void class_map_kernel(const int2* jobs, int n_jobs, const DevLig* ligs,
                                                         int n_small, int32_t* map, uint32_t* queues)
{
    __shared__ int wn0[16], wn1[16];
    const int t = threadIdx.x, w = t / kWave;
    if (t < 2) queues[t] = 0u;
    int base0 = 0, base1 = n_small;
    for (int c = 0; c < n_jobs; c += 1024) {
        const int j = c + t;
        const bool valid = j < n_jobs;
        const bool big = valid && ligs[jobs[j].x].n_atoms > 64;
        const bool small = valid && !big;
        const uint64_t ms = __ballot(small), mb = __ballot(big);
        if ((t & (kWave - 1)) == 0) { wn0[w] = __popcll(ms); wn1[w] = __popcll(mb); }
        __syncthreads();
        int off0 = 0, off1 = 0, tot0 = 0, tot1 = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int a = wn0[q], b = wn1[q];
            off0 += q < w ? a : 0;
            off1 += q < w ? b : 0;
            tot0 += a;
            tot1 += b;
        }
        const int r0 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(ms >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ms, 0u));
        const int r1 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
        if (small) map[base0 + off0 + r0] = j;
        if (big) map[base1 + off1 + r1] = j;
        base0 += tot0;
        base1 += tot1;
        __syncthreads();   // every wave has read wn0 / wn1 before the next chunk writes them
    }
}

hipError_t launch_class_map(const int2* jobs, int32_t n_jobs, const DevLig* ligs, int32_t n_small, int32_t* map,
                            uint32_t* queues, hipStream_t s)
{
    hipLaunchKernelGGL(class_map_kernel, dim3(1), dim3(1024), 0, s, jobs, n_jobs, ligs, n_small, map, queues);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
hipError_t launch_build_grids(const GridBuildArgs& a, int64_t n_tiles, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(gridmap_kernel, dim3((unsigned)n_tiles), dim3(kGridThreads), 0, s, a);
    return hipGetLastError();
}

template <typename K>
static int occupancy(K kernel, int lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, 64, lds) != hipSuccess) return 0;
    return n;
}

template <int A, bool SL>
static int kind_occupancy(int kind, int lds)
{
    if (kind == kKindDock) {   // the fewer of the history capacities' resident blocks
        return std::min(occupancy(dock_kernel<A, SL, kShortM>, lds), occupancy(dock_kernel<A, SL, kMaxM>, lds));
    }
    if (kind == kKindScore) return occupancy(score_kernel<A, SL>, lds);
    return occupancy(local_opt_kernel<A, SL>, lds);
}

// Slots are faster per evaluation but take 16 B per pair end in LDS; they
// are used while the CUs can still hold as many of the launch's waves as the
// gather layout would (a persistent launch over few chains, or small
// ligands), else the gather layout keeps the occupancy.
hipError_t launch_shape(int kind, const LigDev& l, int64_t items, int n_cu, LaunchShape* out)
{
    const int64_t cus = n_cu > 0 ? n_cu : 1;
    if (l.max_atoms > 64) {
        const int lds = lds_bytes(l.max_atoms, l.max_pairs, l.max_ell, kernel_needs(kind, 2, false));
        *out = {2, lds, kind_occupancy<2, false>(kind, lds)};
        return out->per_cu > 0 ? hipSuccess : hipErrorInvalidConfiguration;
    }
    const int lds_s = lds_bytes(l.max_atoms, l.max_pairs, l.max_ell, kernel_needs(kind, 1, true));
    const int lds_g = lds_bytes(l.max_atoms, l.max_pairs, l.max_ell, kernel_needs(kind, 1, false));
    const int occ_s = kind_occupancy<1, true>(kind, lds_s);
    const int occ_g = kind_occupancy<1, false>(kind, lds_g);
    const int64_t need = std::min<int64_t>(items > 0 ? items : 1, (int64_t)occ_g * cus);
    if (occ_s > 0 && (int64_t)occ_s * cus >= need)
        *out = {0, lds_s, occ_s};
    else
        *out = {1, lds_g, occ_g};
    return out->per_cu > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t launch_shape_variant(int kind, const LigDev& l, int variant, LaunchShape* out)
{
    *out = {variant, 0, 0};
    if (variant < 0 || variant > 2 || (variant < 2 && l.max_atoms > 64)) return hipErrorInvalidValue;
    const int lds = lds_bytes(l.max_atoms, l.max_pairs, l.max_ell, kernel_needs(kind, variant == 2 ? 2 : 1, variant == 0));
    int occ;
    if (variant == 0) occ = kind_occupancy<1, true>(kind, lds);
    else if (variant == 1) occ = kind_occupancy<1, false>(kind, lds);
    else occ = kind_occupancy<2, false>(kind, lds);
    *out = {variant, lds, occ};
    return occ > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

hipError_t launch_score(const ScoreArgs& a, int n_cu, hipStream_t s)
{
    if (a.n_poses <= 0) return hipSuccess;
    LaunchShape sh;
    hipError_t e;
    if ((e = launch_shape(kKindScore, a.l, a.n_poses, n_cu, &sh)) != hipSuccess) return e;
    // one resident wave per slot the CUs can hold; each takes a contiguous run
    const int64_t cap = (int64_t)sh.per_cu * (n_cu > 0 ? n_cu : 1);
    const int grid = (int)(a.n_poses < cap ? a.n_poses : cap);
    if (sh.variant == 0)
        hipLaunchKernelGGL((score_kernel<1, true>), dim3(grid), dim3(64), sh.lds, s, a);
    else if (sh.variant == 1)
        hipLaunchKernelGGL((score_kernel<1, false>), dim3(grid), dim3(64), sh.lds, s, a);
    else
        hipLaunchKernelGGL((score_kernel<2, false>), dim3(grid), dim3(64), sh.lds, s, a);
    return hipGetLastError();
}

hipError_t launch_dock(const DockArgs& a, const LaunchShape& sh, int32_t workgroups, hipStream_t s)
{
    if (a.n_items <= 0) return hipSuccess;
    const unsigned grid = a.persistent ? (unsigned)workgroups : (unsigned)a.n_items;
    const bool short_m = a.sp.m <= kShortM;
    if (sh.variant == 0) {
        if (short_m) hipLaunchKernelGGL((dock_kernel<1, true, kShortM>), dim3(grid), dim3(64), sh.lds, s, a);
        else hipLaunchKernelGGL((dock_kernel<1, true, kMaxM>), dim3(grid), dim3(64), sh.lds, s, a);
    } else if (sh.variant == 1) {
        if (short_m) hipLaunchKernelGGL((dock_kernel<1, false, kShortM>), dim3(grid), dim3(64), sh.lds, s, a);
        else hipLaunchKernelGGL((dock_kernel<1, false, kMaxM>), dim3(grid), dim3(64), sh.lds, s, a);
    } else {
        if (short_m) hipLaunchKernelGGL((dock_kernel<2, false, kShortM>), dim3(grid), dim3(64), sh.lds, s, a);
        else hipLaunchKernelGGL((dock_kernel<2, false, kMaxM>), dim3(grid), dim3(64), sh.lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_fma_peak(float* out, int n, int iters, hipStream_t s)
{
    hipLaunchKernelGGL(fma_peak_kernel, dim3((unsigned)(n / 256)), dim3(256), 0, s, out, iters);
    return hipGetLastError();
}

hipError_t launch_reset_queue(uint32_t* q, hipStream_t s)
{
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, q);
    return hipGetLastError();
}

hipError_t launch_reset_times(uint64_t* t0, uint64_t* t1, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(reset_times_kernel, dim3((n + 255) / 256), dim3(256), 0, s, t0, t1, n);
    return hipGetLastError();
}

hipError_t launch_job_reduce(const float* cbe, const int64_t* cev, const int32_t* cst, int32_t n_jobs,
                             int32_t chains, float* jbe, int32_t* jbc, int64_t* jev, int32_t* jst, hipStream_t s)
{
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(job_reduce_kernel, dim3((n_jobs + 255) / 256), dim3(256), 0, s, cbe, cev, cst, n_jobs, chains,
                       jbe, jbc, jev, jst);
    return hipGetLastError();
}

hipError_t launch_local_opt(const OptArgs& a, int n_cu, hipStream_t s)
{
    if (a.n_poses <= 0) return hipSuccess;
    LaunchShape sh;
    hipError_t e;
    if ((e = launch_shape(kKindOpt, a.l, a.n_poses, n_cu, &sh)) != hipSuccess) return e;
    const int grid = a.n_poses < 65536 ? a.n_poses : 65536;
    if (sh.variant == 0)
        hipLaunchKernelGGL((local_opt_kernel<1, true>), dim3(grid), dim3(64), sh.lds, s, a);
    else if (sh.variant == 1)
        hipLaunchKernelGGL((local_opt_kernel<1, false>), dim3(grid), dim3(64), sh.lds, s, a);
    else
        hipLaunchKernelGGL((local_opt_kernel<2, false>), dim3(grid), dim3(64), sh.lds, s, a);
    return hipGetLastError();
}

hipError_t launch_output(const OutputArgs& a, hipStream_t s)
{
    if (a.n_jobs <= 0) return hipSuccess;
    const int lds = output_lds_bytes(a.l, a.chains, a.modes);
    if (a.l.max_atoms <= 64)
        hipLaunchKernelGGL((output_kernel<1>), dim3(a.n_jobs), dim3(64), lds, s, a);
    else
        hipLaunchKernelGGL((output_kernel<2>), dim3(a.n_jobs), dim3(64), lds, s, a);
    return hipGetLastError();
}

int output_lds_bytes(const LigDev& l, int chains, int modes)
{
    const int ma = lds_atoms(l.max_atoms);
    return lds_bytes(l.max_atoms, l.max_pairs, l.max_ell, kernel_needs(kKindOutput, l.max_atoms > 64 ? 2 : 1, false)) +
           round_up(chains, 4) * 4 + modes * ma * 16 +
           modes * kSlot * 4 + 5 * round_up(modes, 4) * 4;
}

hipError_t launch_sas_candidates(const float4* atoms, int n_rec, const float* dirs, int n_dirs, float probe,
                                 int64_t n_cand, float4* cand, uint8_t* keep, int32_t* block_count, hipStream_t s)
{
    if (n_cand <= 0) return hipSuccess;
    const int64_t blocks = (n_cand + kSasThreads - 1) / kSasThreads;
    hipLaunchKernelGGL(sas_candidates_kernel, dim3((unsigned)blocks), dim3(kSasThreads), 0, s, atoms, n_rec, dirs,
                       n_dirs, probe, n_cand, cand, keep, block_count);
    return hipGetLastError();
}

hipError_t launch_sas_scatter(const float4* cand, const uint8_t* keep, const int32_t* block_offset, int64_t n_cand,
                              float4* pts, hipStream_t s)
{
    if (n_cand <= 0) return hipSuccess;
    const int64_t blocks = (n_cand + kSasThreads - 1) / kSasThreads;
    hipLaunchKernelGGL(sas_scatter_kernel, dim3((unsigned)blocks), dim3(kSasThreads), 0, s, cand, keep, block_offset,
                       n_cand, pts);
    return hipGetLastError();
}

hipError_t launch_sas_features(const float4* atoms, int n_rec, const float4* pts, int n_pts, float* feat,
                               hipStream_t s)
{
    if (n_pts <= 0) return hipSuccess;
    const int blocks = (n_pts + kSasThreads - 1) / kSasThreads;
    hipLaunchKernelGGL(sas_features_kernel, dim3(blocks), dim3(kSasThreads), 0, s, atoms, n_rec, pts, n_pts, feat);
    return hipGetLastError();
}

int sas_block_size() { return kSasThreads; }

}  // namespace pv
