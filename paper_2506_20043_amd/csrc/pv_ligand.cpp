// pv_ligand.cpp -- host construction of the ligand model that the kernels
// consume: rigid fragments, the torsion tree in depth-first preorder, the
// atom order that makes every torsion move one contiguous atom range, and
// the intra pair list (the POT of Eq. qvina_eq_1 and the e_intra pairs of
// Eq. qvina_eq_3).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "pv_internal.h"
#include "../../include/pvdock.h"

namespace pv {

namespace {
const double kRadius[kNTypes] = {1.9, 1.9, 1.8, 1.8, 1.8, 1.7, 1.7, 2.0};
const bool kHyd[kNTypes] = {true, false, false, false, false, false, false, false};
const bool kDon[kNTypes] = {false, false, false, true, false, false, true, false};
const bool kAcc[kNTypes] = {false, false, false, false, true, true, true, false};

int find_root(std::vector<int>& up, int a)
{
    while (up[a] != a) {
        up[a] = up[up[a]];
        a = up[a];
    }
    return a;
}
}  // namespace

int build_ligand_model(int n, const float* xyz, const uint8_t* type, int nb, const int32_t* bonds,
                       const uint8_t* rot, LigModel& M, std::string& err)
{
    if (n < 1) { err = "a ligand needs at least one atom"; return PV_E_INVALID; }
    if (n > kMaxAtoms) { err = "ligand has more than 128 atoms"; return PV_E_RANGE; }
    if (nb < n - 1) { err = "ligand is not connected (too few bonds)"; return PV_E_INVALID; }
    for (int i = 0; i < n; ++i) {
        if (type[i] >= kNTypes) { err = "atom type out of range"; return PV_E_INVALID; }
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(xyz[3 * i + a])) { err = "non-finite reference coordinate"; return PV_E_INVALID; }
    }
    std::vector<std::vector<int>> adj(n);
    for (int b = 0; b < nb; ++b) {
        int u = bonds[2 * b], v = bonds[2 * b + 1];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) { err = "bond index out of range or self bond"; return PV_E_INVALID; }
        if (std::find(adj[u].begin(), adj[u].end(), v) != adj[u].end()) { err = "duplicate bond"; return PV_E_INVALID; }
        adj[u].push_back(v);
        adj[v].push_back(u);
    }
    // connectivity
    {
        std::vector<char> seen(n, 0);
        std::vector<int> stack{0};
        seen[0] = 1;
        int cnt = 1;
        while (!stack.empty()) {
            int u = stack.back();
            stack.pop_back();
            for (int v : adj[u])
                if (!seen[v]) { seen[v] = 1; ++cnt; stack.push_back(v); }
        }
        if (cnt != n) { err = "ligand is not connected"; return PV_E_INVALID; }
    }
    // rigid fragments: union-find over non-rotatable bonds
    std::vector<int> up(n);
    std::iota(up.begin(), up.end(), 0);
    int nt = 0;
    for (int b = 0; b < nb; ++b) {
        if (rot[b]) { ++nt; continue; }
        int ru = find_root(up, bonds[2 * b]), rv = find_root(up, bonds[2 * b + 1]);
        if (ru != rv) up[std::max(ru, rv)] = std::min(ru, rv);
    }
    if (nt > kMaxTors) { err = "ligand has more than 32 rotatable bonds"; return PV_E_RANGE; }
    // fragment ids numbered by their lowest atom index
    std::vector<int> fid(n, -1), rep_id(n, -1);
    int nf = 0;
    for (int i = 0; i < n; ++i) {
        int r = find_root(up, i);
        if (rep_id[r] < 0) rep_id[r] = nf++;
        fid[i] = rep_id[r];
    }
    std::vector<int> tors_bond;
    for (int b = 0; b < nb; ++b)
        if (rot[b]) {
            if (fid[bonds[2 * b]] == fid[bonds[2 * b + 1]]) { err = "rotatable bond inside a ring"; return PV_E_INVALID; }
            tors_bond.push_back(b);
        }
    if (nf != nt + 1) { err = "rotatable bonds do not form a tree of fragments"; return PV_E_INVALID; }
    std::vector<int> fsize(nf, 0);
    for (int i = 0; i < n; ++i) fsize[fid[i]]++;
    int root = 0;
    for (int f = 1; f < nf; ++f)
        if (fsize[f] > fsize[root]) root = f;
    // fragment adjacency through torsions
    std::vector<std::vector<int>> ftors(nf);
    for (int k = 0; k < nt; ++k) {
        int b = tors_bond[k];
        ftors[fid[bonds[2 * b]]].push_back(k);
        ftors[fid[bonds[2 * b + 1]]].push_back(k);
    }
    // depth-first preorder from the root; children in torsion order
    std::vector<int> order, parent_of(nf, -1), tors_of(nf, -1), depth_of(nf, 0);
    std::vector<char> visited(nf, 0);
    std::vector<int> stack{root};
    visited[root] = 1;
    while (!stack.empty()) {
        int f = stack.back();
        stack.pop_back();
        order.push_back(f);
        std::vector<std::pair<int, int>> kids;
        for (int k : ftors[f]) {
            int b = tors_bond[k];
            int other = fid[bonds[2 * b]] == f ? fid[bonds[2 * b + 1]] : fid[bonds[2 * b]];
            if (!visited[other]) kids.push_back({k, other});
        }
        // push in reverse so the lowest torsion is visited first
        for (auto it = kids.rbegin(); it != kids.rend(); ++it) {
            visited[it->second] = 1;
            parent_of[it->second] = f;
            tors_of[it->second] = it->first;
            depth_of[it->second] = depth_of[f] + 1;
            stack.push_back(it->second);
        }
    }
    std::vector<int> new_frag(nf);
    for (int i = 0; i < nf; ++i) new_frag[order[i]] = i;
    // atom order: fragments in preorder, atoms ascending inside a fragment
    std::vector<int> perm, inv(n);
    std::vector<int> a0(nf), a1(nf);
    for (int i = 0; i < nf; ++i) {
        a0[i] = (int)perm.size();
        for (int a = 0; a < n; ++a)
            if (fid[a] == order[i]) perm.push_back(a);
        a1[i] = (int)perm.size();
    }
    for (int i = 0; i < n; ++i) inv[perm[i]] = i;
    // subtree size in preorder
    std::vector<int> sub_size(nf, 1);
    for (int i = nf - 1; i > 0; --i) sub_size[new_frag[parent_of[order[i]]]] += sub_size[i];

    M = LigModel();
    M.n = n; M.nf = nf; M.nt = nt; M.root_size = fsize[root];
    M.perm = perm;
    M.ref.resize(4 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        int a = perm[i];
        M.ref[4 * i + 0] = xyz[3 * a + 0];
        M.ref[4 * i + 1] = xyz[3 * a + 1];
        M.ref[4 * i + 2] = xyz[3 * a + 2];
        uint32_t w = (uint32_t)type[a] | ((uint32_t)new_frag[fid[a]] << 8);
        float wf;
        std::memcpy(&wf, &w, 4);
        M.ref[4 * i + 3] = wf;
    }
    M.frags.resize(nf);
    M.tors_frag.assign(nt, 0);
    int maxd = 0;
    for (int i = 0; i < nf; ++i) {
        int f = order[i];
        DevFrag& D = M.frags[i];
        std::memset(&D, 0, sizeof(D));
        D.parent = i == 0 ? -1 : new_frag[parent_of[f]];
        D.tors = tors_of[f];
        D.a0 = a0[i];
        D.sub_end = a1[i + sub_size[i] - 1];
        maxd = std::max(maxd, depth_of[f]);
        if (i == 0) { D.child_atom = -1; continue; }
        int k = tors_of[f], b = tors_bond[k];
        int u = bonds[2 * b], v = bonds[2 * b + 1];
        int c = fid[u] == f ? u : v;     // child side
        int p = c == u ? v : u;          // parent side
        double ax = (double)xyz[3 * c] - xyz[3 * p], ay = (double)xyz[3 * c + 1] - xyz[3 * p + 1],
               az = (double)xyz[3 * c + 2] - xyz[3 * p + 2];
        double nrm = std::sqrt(ax * ax + ay * ay + az * az);
        if (!(nrm > 0.0)) { err = "rotatable bond of zero length"; return PV_E_INVALID; }
        D.axis[0] = (float)(ax / nrm); D.axis[1] = (float)(ay / nrm); D.axis[2] = (float)(az / nrm);
        D.xc[0] = xyz[3 * c]; D.xc[1] = xyz[3 * c + 1]; D.xc[2] = xyz[3 * c + 2];
        D.child_atom = inv[c];
        M.tors_frag[k] = i;
    }
    M.depth = maxd;
    int r = 0;
    while ((1 << r) < maxd + 1) ++r;
    M.rounds = r;
    // anchor: centroid of the root fragment; radius of gyration of all atoms
    double c[3] = {0, 0, 0}, ca[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            ca[a] += xyz[3 * i + a];
            if (fid[i] == root) c[a] += xyz[3 * i + a];
        }
    double s2 = 0;
    for (int a = 0; a < 3; ++a) { c[a] /= fsize[root]; ca[a] /= n; }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) { double d = xyz[3 * i + a] - ca[a]; s2 += d * d; }
    for (int a = 0; a < 3; ++a) M.anchor[a] = (float)c[a];
    M.rg = (float)std::sqrt(s2 / n);
    // intra pairs: breadth-first bond distances from every atom
    std::vector<std::pair<int, int>> pl;
    std::vector<int> dist(n);
    for (int s = 0; s < n; ++s) {
        std::fill(dist.begin(), dist.end(), -1);
        std::vector<int> q{s};
        dist[s] = 0;
        for (size_t h = 0; h < q.size(); ++h)
            for (int v : adj[q[h]])
                if (dist[v] < 0) { dist[v] = dist[q[h]] + 1; q.push_back(v); }
        for (int t = s + 1; t < n; ++t)
            if (fid[s] != fid[t] && dist[t] >= 4) {
                int i = inv[s], j = inv[t];
                pl.push_back({std::min(i, j), std::max(i, j)});
            }
    }
    // pairs grouped by interaction class (plain, hydrophobic, hydrogen bond)
    // so that the class-specific terms are mostly wave-uniform branches
    auto cls = [&](const std::pair<int, int>& q) {
        const int a = type[perm[q.first]], b = type[perm[q.second]];
        if (kHyd[a] && kHyd[b]) return 1;
        if ((kDon[a] && kAcc[b]) || (kAcc[a] && kDon[b])) return 2;
        return 0;
    };
    std::sort(pl.begin(), pl.end(), [&](const std::pair<int, int>& x, const std::pair<int, int>& y) {
        const int cx = cls(x), cy = cls(y);
        return cx != cy ? cx < cy : x < y;
    });
    M.np = (int)pl.size();
    const int P = M.np;
    M.pairs.reserve(P);
    for (int idx = 0; idx < P; ++idx) {
        int i = pl[idx].first, j = pl[idx].second;
        // radius sum 3.4 + 0.1 rk A (every radius is 1.7 + 0.1 k A)
        const int ta = type[perm[i]], tb = type[perm[j]];
        const int rk = (int)std::lround((kRadius[ta] + kRadius[tb] - 3.4) * 10.0);
        M.pairs.push_back((uint32_t)i | ((uint32_t)j << 8) | ((uint32_t)rk << 16) |
                          ((uint32_t)cls(pl[idx]) << 24));
    }
    // atom -> pair rows (partners in ascending pair order), padded to the longest;
    // an entry is the pair index | the partner's byte offset in the kernels'
    // LDS position array (16 B per atom) << 16
    std::vector<std::vector<uint32_t>> rows(n);
    for (int q = 0; q < P; ++q) {
        const uint32_t i = M.pairs[q] & 0xff, j = (M.pairs[q] >> 8) & 0xff;
        rows[i].push_back((uint32_t)q | ((j * 16) << 16));
        rows[j].push_back((uint32_t)q | ((i * 16) << 16));
    }
    int w = 0;
    for (int i = 0; i < n; ++i) w = std::max(w, (int)rows[i].size());
    w = (w + 3) / 4 * 4;   // the kernels read rows four entries at a time
    M.ell_w = w;
    // Slots of the force-slot layout: each pair takes one free slot below w
    // for each of its atoms (any one: an atom sums all its slots).  In LDS
    // slot s of atom a sits at s * (n | 1) + a (float4), and the forces of 16
    // consecutive pairs (an aligned group) are written in one LDS pass per
    // side, so the slots are picked to give each side of a group distinct
    // (s * (n | 1) + a) mod 16: distinct bank groups.
    M.pslot.assign(P, 0u);
    {
        const int stride = n | 1;
        std::vector<uint8_t> used((size_t)n * (w > 0 ? w : 1), 0);
        for (int g0 = 0; g0 < P; g0 += 16) {
            const int g1 = std::min(P, g0 + 16);
            for (int side = 0; side < 2; ++side) {
                uint32_t taken = 0;   // bank groups used by this side of the group
                for (int q = g0; q < g1; ++q) {
                    const int a = side == 0 ? (int)(M.pairs[q] & 0xff) : (int)((M.pairs[q] >> 8) & 0xff);
                    int pick = -1, any = -1;
                    for (int sl = 0; sl < w; ++sl) {
                        if (used[(size_t)a * w + sl]) continue;
                        if (any < 0) any = sl;
                        if (!((taken >> ((sl * stride + a) & 15)) & 1u)) { pick = sl; break; }
                    }
                    if (pick < 0) pick = any;   // a row always has a free slot: w >= its length
                    used[(size_t)a * w + pick] = 1;
                    taken |= 1u << ((pick * stride + a) & 15);
                    M.pslot[q] |= (uint32_t)pick << (16 * side);
                }
            }
        }
    }
    // row-major ([n][w], w a multiple of four): a lane reads four of its
    // atom's entries with one 16-byte load (measured faster than entry-major
    // [w][n] with one load per entry, and than groups of four side by side)
    M.ell.assign((size_t)w * n, 0u);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < w; ++k)
            M.ell[(size_t)i * w + k] =
                k < (int)rows[i].size() ? rows[i][k] : ((uint32_t)P | ((uint32_t)(i * 16) << 16));
    return PV_OK;
}

}  // namespace pv
