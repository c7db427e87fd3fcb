"""FP64 CPU oracle for the nuclear-pasta MD hot path (arXiv:1412.8502).

TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct statement of what
the GPU library computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the HIP
library and never imports the product package.

The arithmetic lives in ``pasta_oracle.c`` (built with gcc, no FMA
contraction).  This module only marshals numpy arrays through ctypes and holds
the paper's constants, restated here independently of the product:

* Table I: a = 110 MeV, b = -26 MeV, c = 24 MeV, Lambda = 1.25 fm^2.
* Screening length fixed to lambda = 10 fm (Sec. II.A, after Eq. 2).
* Nucleon mass M = 939 MeV (Sec. II.A).
* Nuclear cutoff 11.5 fm, no Coulomb cutoff (Sec. II.A, after Eq. 2).
* alpha * hbar c: the paper writes alpha/r in natural units; with CODATA
  alpha = 7.2973525693e-3 and hbar c = 197.3269804 MeV fm it is
  1.4399645 MeV fm.
* Cluster radii r_pp = 4.5 fm and r_np = 3 fm (Sec. II.C).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pasta_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ALPHA = 7.2973525693e-3
HBARC = 197.3269804
PAPER = dict(a=110.0, b=-26.0, c=24.0, Lambda=1.25, lambda_s=10.0,
             alpha_hbarc=ALPHA * HBARC, mass=939.0, r_nuc=11.5,
             r_coul=float("inf"))
R_PP = 4.5
R_NP = 3.0


class _Potential(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("a", "b", "c", "Lambda", "lambda_s", "alpha_hbarc", "mass",
                 "r_nuc", "r_coul")]


class _Integrator(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("xi_dot", ctypes.c_double),
                ("T", ctypes.c_double), ("rescale_every", ctypes.c_int32),
                ("scale_positions", ctypes.c_int32)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
             "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
        vp = ctypes.c_void_p
        lib.oracle_forces.argtypes = [i64, d, vp, vp, P(_Potential), ctypes.c_int,
                                      vp, i64, vp, vp, ctypes.c_int]
        lib.oracle_forces.restype = None
        lib.oracle_pair_counts.argtypes = [i64, d, vp, vp, P(_Potential),
                                           P(i64), P(i64), ctypes.c_int]
        lib.oracle_pair_counts.restype = None
        lib.oracle_run.argtypes = [i64, vp, vp, vp, P(_Potential), P(_Integrator),
                                   d, i64, i64, P(d), P(d), P(d), vp, ctypes.c_int]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_box_length.argtypes = [d, d, d, i64]
        lib.oracle_box_length.restype = d
        lib.oracle_kinetic.argtypes = [i64, vp, d]
        lib.oracle_kinetic.restype = d
        lib.oracle_cluster.argtypes = [i64, d, vp, vp, d, d, vp, P(i32), vp, vp,
                                       P(i32), ctypes.c_int]
        lib.oracle_cluster.restype = ctypes.c_int
        lib.oracle_cell_dims.argtypes = [d, d]
        lib.oracle_cell_dims.restype = ctypes.c_int
        lib.oracle_cell_list.argtypes = [i64, d, d, vp, vp, P(i32), vp, vp]
        lib.oracle_cell_list.restype = ctypes.c_int
        _lib = lib
    return _lib


def _threads(nthreads):
    if nthreads is None:
        nthreads = int(os.environ.get("ORACLE_THREADS", "0")) or (os.cpu_count() or 1)
    return int(nthreads)


def _pot(params=None) -> _Potential:
    p = dict(PAPER)
    if params:
        p.update(params)
    return _Potential(**p)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def forces(pos, species, L, params=None, terms=3, targets=None, nthreads=None):
    """Forces (MeV/fm, [m][3]) and energy shares (MeV, [m]) on `targets`
    (all particles if None).  terms: 1 nuclear, 2 Coulomb, 3 both."""
    lib = _load()
    pos = _c64(pos)
    species = _u8(species)
    n = pos.shape[0]
    if targets is None:
        tptr, m = None, n
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        tptr, m = targets.ctypes.data, targets.shape[0]
    f = np.zeros((m, 3), np.float64)
    e = np.zeros(m, np.float64)
    pot = _pot(params)
    lib.oracle_forces(n, float(L), pos.ctypes.data, species.ctypes.data,
                      ctypes.byref(pot), int(terms), tptr, m, f.ctypes.data,
                      e.ctypes.data, _threads(nthreads))
    return f, e


def pair_counts(pos, species, L, params=None, nthreads=None):
    """(unordered nuclear pairs with r < r_nuc, unordered p-p Coulomb pairs)."""
    lib = _load()
    pos = _c64(pos)
    species = _u8(species)
    a, b = ctypes.c_int64(), ctypes.c_int64()
    pot = _pot(params)
    lib.oracle_pair_counts(pos.shape[0], float(L), pos.ctypes.data, species.ctypes.data,
                           ctypes.byref(pot), ctypes.byref(a), ctypes.byref(b),
                           _threads(nthreads))
    return a.value, b.value


def box_length(L0, xi_dot, dt, step):
    return _load().oracle_box_length(float(L0), float(xi_dot), float(dt), int(step))


def kinetic(vel, mass=PAPER["mass"]):
    vel = _c64(vel)
    return _load().oracle_kinetic(vel.shape[0], vel.ctypes.data, float(mass))


def run(pos, vel, species, L0, nsteps, dt=2.0, xi_dot=0.0, T=1.0, rescale_every=0,
        scale_positions=False, step0=0, params=None, nthreads=None):
    """Velocity-Verlet trajectory.  Returns (pos, vel, L, ekin, epot, force)
    at global step step0 + nsteps; the inputs are not modified."""
    lib = _load()
    pos = _c64(pos).copy()
    vel = _c64(vel).copy()
    species = _u8(species)
    n = pos.shape[0]
    pot = _pot(params)
    integ = _Integrator(dt=float(dt), xi_dot=float(xi_dot), T=float(T),
                        rescale_every=int(rescale_every),
                        scale_positions=int(bool(scale_positions)))
    L, ek, ep = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    f = np.zeros((n, 3), np.float64)
    rc = lib.oracle_run(n, pos.ctypes.data, vel.ctypes.data, species.ctypes.data,
                        ctypes.byref(pot), ctypes.byref(integ), float(L0), int(step0),
                        int(nsteps), ctypes.byref(L), ctypes.byref(ek),
                        ctypes.byref(ep), f.ctypes.data, _threads(nthreads))
    if rc != 0:
        raise MemoryError("oracle_run failed")
    return pos, vel, L.value, ek.value, ep.value, f


def cluster(pos, species, L, r_pp=R_PP, r_np=R_NP, nthreads=None):
    """Cluster algorithm.  Returns dict(label, nclusters, hist_A, hist_Z, nfree)."""
    lib = _load()
    pos = _c64(pos)
    species = _u8(species)
    n = pos.shape[0]
    label = np.zeros(n, np.int32)
    hA = np.zeros(n + 1, np.int32)
    hZ = np.zeros(n + 1, np.int32)
    K, nf = ctypes.c_int32(), ctypes.c_int32()
    rc = lib.oracle_cluster(n, float(L), pos.ctypes.data, species.ctypes.data,
                            float(r_pp), float(r_np), label.ctypes.data,
                            ctypes.byref(K), hA.ctypes.data, hZ.ctypes.data,
                            ctypes.byref(nf), _threads(nthreads))
    if rc != 0:
        raise MemoryError("oracle_cluster failed")
    return dict(label=label, nclusters=K.value, hist_A=hA, hist_Z=hZ, nfree=nf.value)


def cell_dims(L, rcut):
    return _load().oracle_cell_dims(float(L), float(rcut))


def cell_list(pos, species, L, rcut):
    """Returns (ncell, cell_start[2*ncell^3+1], perm[n])."""
    lib = _load()
    pos = _c64(pos)
    species = _u8(species)
    n = pos.shape[0]
    nc = lib.oracle_cell_dims(float(L), float(rcut))
    C = nc ** 3
    start = np.zeros(2 * C + 1, np.int32)
    perm = np.zeros(n, np.int32)
    ncell = ctypes.c_int32()
    rc = lib.oracle_cell_list(n, float(L), float(rcut), pos.ctypes.data,
                              species.ctypes.data, ctypes.byref(ncell),
                              start.ctypes.data, perm.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_cell_list failed")
    return ncell.value, start, perm


def cluster_stats(cl, species, a_min=12):
    """Table II statistics of a cluster result: free-neutron mass fraction,
    and mean and population standard deviation of A and Z over clusters with
    A >= a_min (lighter clusters are left out of the means only)."""
    label = np.asarray(cl["label"])
    species = np.asarray(species)
    K = cl["nclusters"]
    n = label.shape[0]
    A = np.bincount(label[label >= 0], minlength=K)[:K]
    Z = np.bincount(label[(label >= 0) & (species == 1)], minlength=K)[:K]
    heavy = A >= a_min
    out = dict(x_free=cl["nfree"] / n, nclusters=K, n_heavy=int(heavy.sum()))
    if heavy.any():
        out.update(A_mean=float(A[heavy].mean()), A_std=float(A[heavy].std()),
                   Z_mean=float(Z[heavy].mean()), Z_std=float(Z[heavy].std()))
    return out
