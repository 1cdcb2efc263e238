"""Python face of the double-precision CPU oracle (ctypes over libpvoracle.so).

TEST INFRASTRUCTURE ONLY.  The oracle is the checker the HIP path is held to;
only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the product package.

Arrays are numpy; coordinates and pose DOFs are binary64.  Receptor
coordinates are binary32, the interface precision of the receptor; every map
value, including its 8 A cutoff test, is computed from them in binary64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u64p = C.POINTER(C.c_uint64)
_u8p = C.POINTER(C.c_uint8)


class Flags(C.Structure):
    _fields_ = [("min_face", C.c_double), ("min_cut", C.c_double),
                ("min_kink", C.c_double), ("pairs_in", C.c_int64)]


class _Grid(C.Structure):
    _fields_ = [("maps", _dp), ("dims", C.c_int * 3), ("origin", C.c_float * 3),
                ("h", C.c_float), ("kappa", C.c_double)]


class BfgsParams(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("m", C.c_int32), ("ls_max", C.c_int32),
                ("pad", C.c_int32), ("rho", C.c_double), ("sigma", C.c_double),
                ("eps_g", C.c_double), ("eps_c", C.c_double)]


class McParams(C.Structure):
    _fields_ = [("chains", C.c_int32), ("steps", C.c_int32), ("bfgs", BfgsParams),
                ("refine_max_iter", C.c_int32), ("consistency", C.c_int32),
                ("temperature", C.c_double), ("mut_pos_amp", C.c_double),
                ("mut_rot_amp", C.c_double), ("seed", C.c_uint64)]


class BfgsMargins(C.Structure):
    _fields_ = [("armijo", C.c_double), ("wolfe", C.c_double), ("curvature", C.c_double),
                ("descent", C.c_double), ("pose", C.c_double)]


class OutputParams(C.Structure):
    _fields_ = [("modes", C.c_int32), ("refine_max_iter", C.c_int32), ("rmsd_cut", C.c_double),
                ("affinity_w", C.c_double), ("bfgs", BfgsParams)]


EVAL_FN = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                      C.POINTER(C.c_double))


def _declare(L):
    L.or_terms.argtypes = [C.c_double, _dp, _dp]
    L.or_pair.argtypes = [C.c_int, C.c_int, C.c_double, _dp]
    L.or_pair.restype = C.c_double
    L.or_type_params.argtypes = [C.c_int, _dp, _ip, _ip, _ip]
    L.or_weights.argtypes = [_dp]
    L.or_lattice.argtypes = [_dp, _dp, C.c_double, _ip, _fp]
    L.or_build_maps.argtypes = [C.c_int, _fp, _ip, _ip, _fp, C.c_float, _dp, _dp]
    L.or_map_point.argtypes = [C.c_int, _fp, _ip, _ip, _fp, C.c_float,
                               C.c_int, C.c_int, C.c_int, _dp, _dp]
    L.or_retract.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp]
    L.or_trilinear.argtypes = [_dp, _ip, _fp, C.c_float, C.c_double, _dp, _dp, _dp]
    L.or_trilinear.restype = C.c_double
    L.or_ligand_build.argtypes = [C.c_int, _dp, _ip, C.c_int, _ip, _u8p, C.POINTER(C.c_void_p)]
    L.or_ligand_free.argtypes = [C.c_void_p]
    L.or_ligand_info.argtypes = [C.c_void_p, _ip]
    L.or_ligand_pairs.argtypes = [C.c_void_p, _ip]
    L.or_ligand_frag.argtypes = [C.c_void_p, _ip]
    L.or_ligand_torsions.argtypes = [C.c_void_p, _ip]
    L.or_ligand_rg.argtypes = [C.c_void_p]
    L.or_ligand_rg.restype = C.c_double
    L.or_ligand_anchor.argtypes = [C.c_void_p, _dp]
    L.or_fk.argtypes = [C.c_void_p, _dp, _dp]
    L.or_score_grad.argtypes = [C.c_void_p, C.POINTER(_Grid), _dp, _dp, _dp, _dp, _dp, _dp,
                                C.POINTER(Flags)]
    L.or_score_xyz.argtypes = [C.c_void_p, C.POINTER(_Grid), _dp, _dp, _dp, C.POINTER(Flags)]
    L.or_inter_pairwise.argtypes = [C.c_int, _fp, _ip, C.c_int, _dp, _ip]
    L.or_inter_pairwise.restype = C.c_double
    L.or_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    L.or_bfgs.argtypes = [C.c_void_p, C.POINTER(_Grid), C.POINTER(BfgsParams), _dp, _dp, _dp,
                          _i64p, _ip]
    L.or_bfgs_margins_run.argtypes = [C.c_void_p, C.POINTER(_Grid), C.POINTER(BfgsParams), _dp, _dp, _dp,
                                      _i64p, _ip, C.POINTER(BfgsMargins)]
    L.or_bfgs_generic.argtypes = [C.c_int, EVAL_FN, C.c_void_p, C.POINTER(BfgsParams), _dp, _dp,
                                  _dp, _i64p, _ip]
    L.or_init_pose.argtypes = [C.c_void_p, C.POINTER(_Grid), C.c_uint64, C.c_int, C.c_int, _dp]
    L.or_mc_chain.argtypes = [C.c_void_p, C.POINTER(_Grid), C.POINTER(McParams), C.c_int,
                              C.c_int, _dp, _dp, _i64p]
    L.or_mutate.argtypes = [C.c_void_p, C.POINTER(McParams), _u64p, _dp]
    L.or_metropolis_accepts.argtypes = [C.c_double, C.c_double, C.c_uint64, C.c_double]
    L.or_metropolis_accepts.restype = C.c_int
    L.or_dock.argtypes = [C.c_int, C.POINTER(C.c_void_p), C.c_int, C.POINTER(_Grid), C.c_int,
                          _ip, C.POINTER(McParams), C.c_int, C.c_int, _dp, _dp, _i64p, _dp, _ip]
    L.or_consistency_passes.argtypes = [C.c_int, _dp, C.c_double, _dp, _dp, C.c_double, _dp, C.c_int, C.c_int]
    L.or_sas_points.argtypes = [C.c_int, _fp, _ip, C.c_int, _fp, C.c_float, C.c_int, _fp, _ip]
    L.or_point_features.argtypes = [C.c_int, _fp, _ip, C.c_int, _fp, _dp]
    L.or_output_stage.argtypes = [C.c_void_p, C.POINTER(_Grid), C.c_int, _dp, _dp, C.POINTER(OutputParams),
                                  _ip, _ip, _dp, _dp, _dp, _dp]


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------- terms
def terms(d: float):
    v = np.zeros(5)
    dv = np.zeros(5)
    lib().or_terms(float(d), _p(v, _dp), _p(dv, _dp))
    return v, dv


def pair(ta: int, tb: int, r: float):
    de = C.c_double()
    e = lib().or_pair(int(ta), int(tb), float(r), C.byref(de))
    return e, de.value


def type_params(t: int):
    r = C.c_double()
    h, d, a = C.c_int32(), C.c_int32(), C.c_int32()
    lib().or_type_params(int(t), C.byref(r), C.byref(h), C.byref(d), C.byref(a))
    return r.value, h.value, d.value, a.value


def weights():
    w = np.zeros(5)
    lib().or_weights(_p(w, _dp))
    return w


# ---------------------------------------------------------------- lattice / maps
def lattice(center, size, h):
    c = _f64(center)
    s = _f64(np.broadcast_to(np.asarray(size, dtype=np.float64), (3,)))
    dims = np.zeros(3, np.int32)
    org = np.zeros(3, np.float32)
    rc = lib().or_lattice(_p(c, _dp), _p(s, _dp), float(h), _p(dims, _ip), _p(org, _fp))
    if rc != 0:
        raise ValueError("invalid box (code %d)" % rc)
    return dims, org


def build_maps(rec_xyz, rec_type, dims, origin, h, margin=False):
    """Maps [8][nz][ny][nx]; with margin=True also [nz][ny][nx], per point the
    smallest |r - 8| over the receptor atoms (inf when none is near)."""
    x = _f32(rec_xyz)
    t = _i32(rec_type)
    d = _i32(dims)
    o = _f32(origin)
    out = np.zeros((8, int(d[2]), int(d[1]), int(d[0])), np.float64)
    mg = np.zeros(out.shape[1:], np.float64) if margin else None
    rc = lib().or_build_maps(len(t), _p(x, _fp), _p(t, _ip), _p(d, _ip), _p(o, _fp),
                             float(np.float32(h)), _p(out, _dp), _p(mg, _dp) if margin else None)
    if rc != 0:
        raise ValueError("invalid receptor (code %d)" % rc)
    return (out, mg) if margin else out


def map_point(rec_xyz, rec_type, dims, origin, h, i, j, k, margin=False):
    """The 8 map values at lattice point (i, j, k); with margin=True also the
    smallest |r - 8| over the receptor atoms."""
    x = _f32(rec_xyz)
    t = _i32(rec_type)
    d = _i32(dims)
    o = _f32(origin)
    out = np.zeros(8)
    mg = C.c_double()
    rc = lib().or_map_point(len(t), _p(x, _fp), _p(t, _ip), _p(d, _ip), _p(o, _fp),
                            float(np.float32(h)), int(i), int(j), int(k), _p(out, _dp), C.byref(mg))
    if rc != 0:
        raise ValueError("invalid point (code %d)" % rc)
    return (out, mg.value) if margin else out


def retract(nt, x, d, lam):
    """x (+) lam d, the pose update of the oracle's BFGS."""
    xx = _f64(x)
    dd = _f64(d)
    assert len(xx) == 7 + nt and len(dd) == 6 + nt
    o = np.zeros(7 + nt)
    lib().or_retract(int(nt), _p(xx, _dp), _p(dd, _dp), float(lam), _p(o, _dp))
    return o


class Grid:
    """Maps of one box in binary64 plus its lattice and penalty slope."""

    def __init__(self, maps, dims, origin, h, kappa=1000.0):
        self.maps = _f64(maps)
        self.dims = _i32(dims)
        self.origin = _f32(origin)
        self.h = float(np.float32(h))
        self.kappa = float(kappa)
        self._s = _Grid()
        self._s.maps = _p(self.maps, _dp)
        for a in range(3):
            self._s.dims[a] = int(self.dims[a])
            self._s.origin[a] = float(self.origin[a])
        self._s.h = self.h
        self._s.kappa = self.kappa

    @classmethod
    def build(cls, rec_xyz, rec_type, center, size, h, kappa=1000.0):
        dims, org = lattice(center, size, h)
        return cls(build_maps(rec_xyz, rec_type, dims, org, h), dims, org, h, kappa)

    @property
    def struct(self):
        return self._s

    def trilinear(self, t, x):
        g = np.zeros(3)
        fd = C.c_double()
        xx = _f64(x)
        msz = int(np.prod(self.dims))
        sub = self.maps.reshape(8, msz)[int(t)]
        v = lib().or_trilinear(_p(sub, _dp), _p(self.dims, _ip), _p(self.origin, _fp),
                               self.h, self.kappa, _p(xx, _dp), _p(g, _dp), C.byref(fd))
        return v, g, fd.value


# ---------------------------------------------------------------- ligand
class Ligand:
    def __init__(self, ref_xyz, types, bonds, rotatable):
        self.ref = _f64(ref_xyz).reshape(-1, 3)
        self.types = _i32(types)
        self.bonds = _i32(bonds).reshape(-1, 2)
        self.rot = np.ascontiguousarray(rotatable, dtype=np.uint8)
        h = C.c_void_p()
        rc = lib().or_ligand_build(len(self.types), _p(self.ref, _dp), _p(self.types, _ip),
                                   len(self.bonds), _p(self.bonds, _ip), _p(self.rot, _u8p),
                                   C.byref(h))
        if rc != 0:
            raise ValueError("invalid ligand (code %d)" % rc)
        self.h = h
        info = np.zeros(8, np.int32)
        lib().or_ligand_info(self.h, _p(info, _ip))
        self.n_atoms, self.n_frag, self.n_tors, self.n_pairs, self.root, self.depth = \
            [int(v) for v in info[:6]]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_ligand_free(self.h)
            self.h = None

    @property
    def ndof(self):
        return 7 + self.n_tors

    def pairs(self):
        p = np.zeros((self.n_pairs, 2), np.int32)
        lib().or_ligand_pairs(self.h, _p(p, _ip))
        return p

    def frag(self):
        f = np.zeros(self.n_atoms, np.int32)
        lib().or_ligand_frag(self.h, _p(f, _ip))
        return f

    def torsions(self):
        t = np.zeros((self.n_tors, 3), np.int32)
        lib().or_ligand_torsions(self.h, _p(t, _ip))
        return t

    def rg(self):
        return lib().or_ligand_rg(self.h)

    def anchor(self):
        a = np.zeros(3)
        lib().or_ligand_anchor(self.h, _p(a, _dp))
        return a

    def fk(self, dof):
        d = _f64(dof)
        x = np.zeros((self.n_atoms, 3))
        lib().or_fk(self.h, _p(d, _dp), _p(x, _dp))
        return x

    def score_grad(self, grid: Grid, dof):
        d = _f64(dof)
        e3 = np.zeros(3)
        gd = np.zeros(self.ndof)
        gt = np.zeros(6 + self.n_tors)
        x = np.zeros((self.n_atoms, 3))
        gx = np.zeros((self.n_atoms, 3))
        fl = Flags()
        lib().or_score_grad(self.h, C.byref(grid.struct), _p(d, _dp), _p(e3, _dp), _p(gd, _dp),
                            _p(gt, _dp), _p(x, _dp), _p(gx, _dp), C.byref(fl))
        return dict(e=e3[0], e_inter=e3[1], e_intra=e3[2], grad_dof=gd, grad_tan=gt, xyz=x,
                    grad_xyz=gx, min_face=fl.min_face, min_cut=fl.min_cut,
                    min_kink=fl.min_kink, pairs_in=fl.pairs_in)

    def score_xyz(self, grid: Grid, xyz):
        x = _f64(xyz).reshape(-1, 3)
        e3 = np.zeros(3)
        gx = np.zeros((self.n_atoms, 3))
        fl = Flags()
        lib().or_score_xyz(self.h, C.byref(grid.struct), _p(x, _dp), _p(e3, _dp), _p(gx, _dp),
                           C.byref(fl))
        return dict(e=e3[0], e_inter=e3[1], e_intra=e3[2], grad_xyz=gx, min_face=fl.min_face,
                    min_cut=fl.min_cut, min_kink=fl.min_kink, pairs_in=fl.pairs_in)


def inter_pairwise(rec_xyz, rec_type, xyz, types):
    r = _f32(rec_xyz)
    rt = _i32(rec_type)
    x = _f64(xyz)
    t = _i32(types)
    return lib().or_inter_pairwise(len(rt), _p(r, _fp), _p(rt, _ip), len(t), _p(x, _dp),
                                   _p(t, _ip))


# ---------------------------------------------------------------- RNG
def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64_10(_p(c, _u64p), _p(k, _u64p), _p(out, _u64p))
    return out


# ---------------------------------------------------------------- search
def bfgs_params(max_iter=30, m=5, ls_max=10, rho=1e-4, sigma=0.1, eps_g=1e-3, eps_c=1e-6):
    return BfgsParams(int(max_iter), int(m), int(ls_max), 0, float(rho), float(sigma),
                      float(eps_g), float(eps_c))


def mc_params(chains, steps, seed, bfgs=None, refine_max_iter=None, temperature=1.2,
              mut_pos_amp=2.0, mut_rot_amp=2.0, consistency=False):
    b = bfgs if bfgs is not None else bfgs_params()
    return McParams(int(chains), int(steps), b,
                    int(b.max_iter if refine_max_iter is None else refine_max_iter), int(bool(consistency)),
                    float(temperature), float(mut_pos_amp), float(mut_rot_amp),
                    int(seed) & 0xFFFFFFFFFFFFFFFF)


def bfgs(lig: Ligand, grid: Grid, x0, params: BfgsParams | None = None):
    P = params if params is not None else bfgs_params()
    x = _f64(x0)
    xo = np.zeros(lig.ndof)
    f = C.c_double()
    ne = C.c_int64()
    it = C.c_int32()
    lib().or_bfgs(lig.h, C.byref(grid.struct), C.byref(P), _p(x, _dp), _p(xo, _dp), C.byref(f),
                  C.byref(ne), C.byref(it))
    return xo, f.value, ne.value, it.value


def bfgs_margins(lig: Ligand, grid: Grid, x0, params: BfgsParams | None = None):
    """or_bfgs plus the margins of its decisions: (x, f, n_evals, n_iters,
    {armijo, wolfe, curvature, descent, pose})."""
    P = params if params is not None else bfgs_params()
    x = _f64(x0)
    xo = np.zeros(lig.ndof)
    f = C.c_double()
    ne = C.c_int64()
    it = C.c_int32()
    m = BfgsMargins()
    lib().or_bfgs_margins_run(lig.h, C.byref(grid.struct), C.byref(P), _p(x, _dp), _p(xo, _dp), C.byref(f),
                              C.byref(ne), C.byref(it), C.byref(m))
    return xo, f.value, ne.value, it.value, {k: getattr(m, k) for k, _ in BfgsMargins._fields_}


def bfgs_generic(fun, x0, params: BfgsParams | None = None):
    """The oracle's BFGS on a flat objective: fun(x) -> (f, grad)."""
    P = params if params is not None else bfgs_params()
    x0 = _f64(x0)
    n = len(x0)

    def cb(_user, xp, fp, gp):
        x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
        f, g = fun(x)
        fp[0] = float(f)
        for i in range(n):
            gp[i] = float(g[i])

    cfun = EVAL_FN(cb)
    xo = np.zeros(n)
    f = C.c_double()
    ne = C.c_int64()
    it = C.c_int32()
    lib().or_bfgs_generic(n, cfun, None, C.byref(P), _p(x0, _dp), _p(xo, _dp), C.byref(f),
                          C.byref(ne), C.byref(it))
    return xo, f.value, ne.value, it.value


def init_pose(lig: Ligand, grid: Grid, seed, job, chain):
    d = np.zeros(lig.ndof)
    lib().or_init_pose(lig.h, C.byref(grid.struct), int(seed) & 0xFFFFFFFFFFFFFFFF, int(job),
                       int(chain), _p(d, _dp))
    return d


def mutate(lig: Ligand, params: McParams, words, x):
    """One mutation (Eq. qvina_eq_2) of pose x from the step's 8 Philox words."""
    w = np.ascontiguousarray(words, dtype=np.uint64)
    assert w.shape == (8,)
    y = _f64(x).copy()
    assert len(y) == lig.ndof
    lib().or_mutate(lig.h, C.byref(params), _p(w, _u64p), _p(y, _dp))
    return y


def metropolis_accepts(e_cur, e_new, word, temperature=1.2):
    """The Monte Carlo step's acceptance decision (Eq. qvina_eq_13)."""
    return bool(lib().or_metropolis_accepts(float(e_cur), float(e_new), int(word) & 0xFFFFFFFFFFFFFFFF,
                                            float(temperature)))


def mc_chain(lig: Ligand, grid: Grid, params: McParams, job, chain):
    d = np.zeros(lig.ndof)
    e = C.c_double()
    ne = C.c_int64()
    lib().or_mc_chain(lig.h, C.byref(grid.struct), C.byref(params), int(job), int(chain),
                      _p(d, _dp), C.byref(e), C.byref(ne))
    return d, e.value, ne.value


def dock(ligands, grids, jobs, params: McParams, dof_stride=None, n_threads=0):
    """Every (job, chain) of Supplementary Algorithm 2; jobs = [(ligand, grid)]."""
    jobs = _i32(jobs).reshape(-1, 2)
    nj = len(jobs)
    stride = dof_stride or max(l.ndof for l in ligands)
    hs = (C.c_void_p * len(ligands))(*[l.h for l in ligands])
    gs = (_Grid * len(grids))(*[g.struct for g in grids])
    ch = params.chains
    cbe = np.zeros(nj * ch)
    cbd = np.zeros((nj * ch, stride))
    cev = np.zeros(nj * ch, np.int64)
    jbe = np.zeros(nj)
    jbc = np.zeros(nj, np.int32)
    rc = lib().or_dock(len(ligands), hs, len(grids), gs, nj, _p(jobs, _ip), C.byref(params),
                       int(stride), int(n_threads), _p(cbe, _dp), _p(cbd, _dp), _p(cev, _i64p),
                       _p(jbe, _dp), _p(jbc, _ip))
    if rc != 0:
        raise ValueError("invalid dock input (code %d)" % rc)
    return dict(chain_best_e=cbe.reshape(nj, ch), chain_best_dof=cbd.reshape(nj, ch, stride),
                chain_evals=cev.reshape(nj, ch), job_best_e=jbe, job_best_chain=jbc)


def output_stage(lig: Ligand, grid: Grid, dof, e, modes=20, refine_max_iter=0, rmsd_cut=1.0,
                 affinity_w=0.0585, bfgs=None):
    """The output stage of one job: cluster and sort the chains' best poses
    dof [n][7+T] with energies e [n], refine and rescore the kept ones, then
    r.m.s.d.-filter and sort (see or_output_stage)."""
    d = _f64(np.asarray(dof, dtype=np.float64).reshape(-1, lig.ndof))
    ee = _f64(e).reshape(-1)
    n = len(ee)
    assert d.shape[0] == n
    P = OutputParams(int(modes), int(refine_max_iter), float(rmsd_cut), float(affinity_w),
                     bfgs if bfgs is not None else bfgs_params())
    no = C.c_int32()
    ch = np.zeros(modes, np.int32)
    oe = np.zeros(modes)
    oa = np.zeros(modes)
    od = np.zeros((modes, lig.ndof))
    mg = np.zeros(2)
    rc = lib().or_output_stage(lig.h, C.byref(grid.struct), n, _p(d, _dp), _p(ee, _dp), C.byref(P), C.byref(no),
                               _p(ch, _ip), _p(oe, _dp), _p(oa, _dp), _p(od, _dp), _p(mg, _dp))
    if rc != 0:
        raise ValueError("invalid output-stage input (code %d)" % rc)
    k = no.value
    return {"chain": ch[:k], "e": oe[:k], "affinity": oa[:k], "dof": od[:k], "rmsd_margin": mg[0],
            "energy_gap": mg[1]}


def consistency_passes(nt, x, fx, gx, y, fy, gy, p_lo=0, p_hi=None):
    """The first-order consistency check of a mutated pose x against its
    neighbour y over tangent coordinates [p_lo, p_hi) (or_consistency_passes)."""
    xa, ya, gxa, gya = _f64(x), _f64(y), _f64(gx), _f64(gy)
    hi = 6 + int(nt) if p_hi is None else int(p_hi)
    return bool(lib().or_consistency_passes(int(nt), _p(xa, _dp), float(fx), _p(gxa, _dp), _p(ya, _dp), float(fy),
                                            _p(gya, _dp), int(p_lo), hi))


def sas_points(rec_xyz, rec_type, dirs, probe=1.6):
    """Surface points (binary32 [n][3]) and their atom, see or_sas_points."""
    x = _f32(rec_xyz)
    t = _i32(rec_type)
    d = _f32(dirs)
    cap = max(len(t) * (d.size // 3), 1)
    pts = np.zeros((cap, 3), np.float32)
    atom = np.zeros(cap, np.int32)
    n = lib().or_sas_points(len(t), _p(x, _fp), _p(t, _ip), d.size // 3, _p(d, _fp), float(np.float32(probe)), cap,
                            _p(pts, _fp), _p(atom, _ip))
    if n < 0:
        raise ValueError("invalid surface input")
    return pts[:n].copy(), atom[:n].copy()


def point_features(rec_xyz, rec_type, pts):
    """Eq. prank_eq_1 features and protrusion per point [n][12]."""
    x = _f32(rec_xyz)
    t = _i32(rec_type)
    p = _f32(pts)
    out = np.zeros((p.size // 3, 12))
    lib().or_point_features(len(t), _p(x, _fp), _p(t, _ip), p.size // 3, _p(p, _fp), _p(out, _dp))
    return out
