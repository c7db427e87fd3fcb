"""ctypes binding of libpasta (include/pasta.h).

Argument marshalling only: every computation runs in the HIP library.  torch
supplies device memory (tensors, workspaces) and the stream; the functions
below carry the same names as the C entry points and take torch tensors in
place of raw device pointers.  If libpasta.so has not been built, importing
this module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpasta.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pasta.h")

PASTA_OK = 0
PASTA_EDEVICE = -5
PASTA_FP64 = 0
PASTA_MIXED = 1
PASTA_TERM_NUCLEAR = 1
PASTA_TERM_COULOMB = 2
PASTA_TERM_ALL = 3
PASTA_KERNEL_CLASSES = 9
ERRORS = {-1: "PASTA_EINVAL", -2: "PASTA_EBOX", -3: "PASTA_EWORKSPACE", -4: "PASTA_EHIP",
          -5: "PASTA_EDEVICE", -6: "PASTA_ENOMEM"}


class PastaError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code


class pasta_potential(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("a", "b", "c", "Lambda", "lambda_s", "alpha_hbarc", "mass", "r_nuc",
                 "r_coul")]


class pasta_tuning(ctypes.Structure):
    _fields_ = [("nuclear_variant", ctypes.c_int32), ("coulomb_splits", ctypes.c_int32),
                ("fused_forces", ctypes.c_int32), ("coulomb_form", ctypes.c_int32),
                ("list_skin", ctypes.c_double), ("list_pool_scale", ctypes.c_double),
                ("batch_wgs_per_cu", ctypes.c_int32), ("nuclear_tile", ctypes.c_int32)]


TUNING_FIELDS = ("nuclear_variant", "coulomb_splits", "fused_forces", "coulomb_form",
                 "list_skin", "list_pool_scale", "batch_wgs_per_cu", "nuclear_tile")


class pasta_integrator(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("xi_dot", ctypes.c_double), ("T", ctypes.c_double),
                ("rescale_every", ctypes.c_int32), ("scale_positions", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1412_8502_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, d, i32, i64, sz = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                           ctypes.c_size_t)
    pot, integ = P(pasta_potential), P(pasta_integrator)
    sig = {
        "pasta_potential_paper": (None, [pot]),
        "pasta_set_tuning": (ctypes.c_int, [P(pasta_tuning)]),
        "pasta_autotune_workspace": (ctypes.c_int, [pot, i32, i64, d, P(sz)]),
        "pasta_autotune": (ctypes.c_int, [pot, i32, i64, d, vp, vp, vp, sz, vp, i32,
                                          P(pasta_tuning), vp, vp, P(i32)]),
        "pasta_get_tuning": (ctypes.c_int, [P(pasta_tuning)]),
        "pasta_last_error": (ctypes.c_char_p, []),
        "pasta_version": (ctypes.c_char_p, []),
        "pasta_cell_list_workspace": (ctypes.c_int, [i64, d, d, P(sz)]),
        "pasta_cell_dims": (ctypes.c_int, [d, d, P(i32)]),
        "pasta_cell_list": (ctypes.c_int, [i64, d, d, vp, vp, vp, vp, P(i32), vp, sz, vp]),
        "pasta_forces_workspace": (ctypes.c_int, [pot, i32, i64, d, P(sz)]),
        "pasta_forces": (ctypes.c_int, [pot, i32, i32, i64, d, vp, vp, vp, vp, vp, sz, vp]),
        "pasta_forces_noalloc": (ctypes.c_int, [pot, i32, i32, i64, d, vp, vp, vp, vp, vp]),
        "pasta_sim_workspace": (ctypes.c_int, [pot, integ, i32, i64, d, d, P(sz)]),
        "pasta_sim_create": (ctypes.c_int, [pot, integ, i32, i64, d, i64, d, vp, vp, vp, vp,
                                            sz, vp, P(vp)]),
        "pasta_sim_step": (ctypes.c_int, [vp, i64]),
        "pasta_sim_energies": (ctypes.c_int, [vp, P(d), P(d), P(d), P(i64)]),
        "pasta_sim_forces": (ctypes.c_int, [vp, vp, vp]),
        "pasta_sim_pair_counts": (ctypes.c_int, [vp, P(i64), P(i64)]),
        "pasta_sim_get_step": (ctypes.c_int, [vp, P(i64)]),
        "pasta_sim_get_state": (ctypes.c_int, [vp, vp, vp, P(i64)]),
        "pasta_sim_set_state": (ctypes.c_int, [vp, vp, vp, i64]),
        "pasta_sim_set_timing": (ctypes.c_int, [vp, i32]),
        "pasta_sim_kernel_times": (ctypes.c_int, [vp, vp, vp]),
        "pasta_kernel_class_name": (ctypes.c_char_p, [i32]),
        "pasta_sim_list_stats": (ctypes.c_int, [vp, P(i64), P(i64), P(d), P(i64), P(i64)]),
        "pasta_sim_destroy": (None, [vp]),
        "pasta_cluster_workspace": (ctypes.c_int, [i64, d, d, d, P(sz)]),
        "pasta_batch_workspace": (ctypes.c_int, [pot, i32, i32, vp, vp, P(sz)]),
        "pasta_batch_create": (ctypes.c_int, [pot, i32, i32, vp, vp, vp, i64, vp, vp, vp, vp,
                                              vp, sz, i32, i32, vp, P(vp)]),
        "pasta_batch_step": (ctypes.c_int, [vp, i64]),
        "pasta_batch_set_wait_limit": (ctypes.c_int, [vp, i64]),
        "pasta_batch_energies": (ctypes.c_int, [vp, vp, vp, vp, P(i64)]),
        "pasta_batch_forces": (ctypes.c_int, [vp, vp, vp]),
        "pasta_batch_pair_counts": (ctypes.c_int, [vp, vp, vp]),
        "pasta_batch_info": (ctypes.c_int, [vp, P(i32), P(i32)]),
        "pasta_batch_destroy": (None, [vp]),
        "pasta_cluster": (ctypes.c_int, [i64, d, vp, vp, d, d, vp, vp, vp, P(i32), P(i32), vp,
                                         sz, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def header_functions():
    """Names of the functions declared in include/pasta.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pasta_[a-z0-9_]+)\s*\(", text)))


def _check(rc: int):
    if rc != PASTA_OK:
        raise PastaError(rc, lib.pasta_last_error().decode())


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes: int, device):
    # 256-byte aligned: the caching allocator returns 512-byte aligned blocks
    w = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert w.data_ptr() % 256 == 0
    return w


def _check_state(pos, species):
    if pos.dtype != torch.float64 or pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_cuda:
        raise ValueError("pos must be a CUDA float64 tensor of shape [n, 3]")
    if species.dtype != torch.uint8 or species.shape != (pos.shape[0],) or not species.is_cuda:
        raise ValueError("species must be a CUDA uint8 tensor of shape [n]")
    if not (pos.is_contiguous() and species.is_contiguous()):
        raise ValueError("pos and species must be contiguous")


def pasta_potential_paper() -> pasta_potential:
    p = pasta_potential()
    lib.pasta_potential_paper(ctypes.byref(p))
    return p


def tuning_dict(t: pasta_tuning) -> dict:
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def pasta_get_tuning() -> dict:
    cur = pasta_tuning()
    _check(lib.pasta_get_tuning(ctypes.byref(cur)))
    return tuning_dict(cur)


def pasta_set_tuning(**kw):
    """Process-wide kernel choices (see pasta_tuning in include/pasta.h):
    any of nuclear_variant, coulomb_splits, fused_forces, coulomb_form,
    list_skin, list_pool_scale; the others keep their values.  Returns the previous
    setting as a dict."""
    bad = set(kw) - set(TUNING_FIELDS)
    if bad:
        raise TypeError(f"unknown tuning fields {sorted(bad)}")
    old = pasta_get_tuning()
    merged = dict(old)
    merged.update({k: v for k, v in kw.items() if v is not None})
    new = pasta_tuning()
    for f in TUNING_FIELDS:
        setattr(new, f, merged[f])
    _check(lib.pasta_set_tuning(ctypes.byref(new)))
    return old


def pasta_version() -> str:
    return lib.pasta_version().decode()


def pasta_kernel_class_name(k: int) -> str:
    return lib.pasta_kernel_class_name(k).decode()


# ------------------------------------------------------------------- a1
def pasta_cell_list(pos, species, L: float, r_cut: float, stream=None):
    """Returns (ncell, cell_start int32 [2 ncell^3 + 1], perm int32 [n])."""
    _check_state(pos, species)
    n = pos.shape[0]
    nb = ctypes.c_size_t()
    _check(lib.pasta_cell_list_workspace(n, L, r_cut, ctypes.byref(nb)))
    work = _workspace(nb.value, pos.device)
    dims = ctypes.c_int32()
    _check(lib.pasta_cell_dims(L, r_cut, ctypes.byref(dims)))
    nc = dims.value
    start = torch.empty(2 * nc ** 3 + 1, dtype=torch.int32, device=pos.device)
    perm = torch.empty(n, dtype=torch.int32, device=pos.device)
    ncell = ctypes.c_int32()
    _check(lib.pasta_cell_list(n, L, r_cut, _p(pos), _p(species), _p(start), _p(perm),
                               ctypes.byref(ncell), _p(work), work.numel(), _stream(stream)))
    assert ncell.value == nc
    return nc, start, perm


# -------------------------------------------------------------- a2 + a3
def pasta_forces(pos, species, L: float, precision: int = PASTA_FP64,
                 terms: int = PASTA_TERM_ALL, pot: pasta_potential | None = None,
                 stream=None):
    """Returns (force float64 [n, 3], epot float64 [n])."""
    _check_state(pos, species)
    pot = pot or pasta_potential_paper()
    n = pos.shape[0]
    nb = ctypes.c_size_t()
    _check(lib.pasta_forces_workspace(ctypes.byref(pot), precision, n, L, ctypes.byref(nb)))
    work = _workspace(nb.value, pos.device)
    force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    epot = torch.empty(n, dtype=torch.float64, device=pos.device)
    _check(lib.pasta_forces(ctypes.byref(pot), precision, terms, n, L, _p(pos), _p(species),
                            _p(force), _p(epot), _p(work), work.numel(), _stream(stream)))
    return force, epot


def pasta_forces_noalloc(pos, species, L: float, force, epot=None,
                         precision: int = PASTA_FP64, terms: int = PASTA_TERM_ALL,
                         pot: pasta_potential | None = None, stream=None):
    """pasta_forces into caller tensors (force float64 [n, 3], epot float64
    [n] or None) with the library's static scratch: no workspace."""
    _check_state(pos, species)
    pot = pot or pasta_potential_paper()
    n = pos.shape[0]
    for t, shape in ((force, (n, 3)), (epot, (n,))):
        if t is not None and (t.shape != shape or t.dtype != torch.float64 or
                              not t.is_contiguous() or t.device != pos.device):
            raise ValueError("force / epot must be contiguous float64 tensors on pos's device")
    _check(lib.pasta_forces_noalloc(ctypes.byref(pot), precision, terms, n, L, _p(pos),
                                    _p(species), _p(force), _p(epot),
                                    _stream(stream)))
    return force, epot


# ------------------------------------------------------------------- a4
class Sim:
    """Owner of a pasta_sim handle and of its workspace tensor.  The library
    keeps the state in sorted order; `pos` and `vel` receive the current
    state after every `step` call (stream order) and are read again only by
    `set_state`."""

    def __init__(self, pos, vel, species, L0: float, dt: float = 2.0, xi_dot: float = 0.0,
                 T: float = 1.0, rescale_every: int = 0, scale_positions: bool = False,
                 precision: int = PASTA_FP64, step0: int = 0, L_max: float | None = None,
                 pot: pasta_potential | None = None, stream=None):
        _check_state(pos, species)
        if vel.shape != pos.shape or vel.dtype != torch.float64 or not vel.is_contiguous():
            raise ValueError("vel must be a contiguous float64 tensor shaped like pos")
        self.pos, self.vel, self.species = pos, vel, species
        self.pot = pot or pasta_potential_paper()
        self.integ = pasta_integrator(dt, xi_dot, T, rescale_every, int(bool(scale_positions)))
        self.precision = precision
        self.n = pos.shape[0]
        self.stream = stream
        if L_max is None:
            L_max = L0
        L_start = L0 * (1.0 + xi_dot * step0 * dt)
        nb = ctypes.c_size_t()
        _check(lib.pasta_sim_workspace(ctypes.byref(self.pot), ctypes.byref(self.integ),
                                       precision, self.n, L_start, max(L_max, L_start),
                                       ctypes.byref(nb)))
        self.work = _workspace(nb.value, pos.device)
        self.handle = ctypes.c_void_p()
        _check(lib.pasta_sim_create(ctypes.byref(self.pot), ctypes.byref(self.integ), precision,
                                    self.n, L0, step0, L_max, _p(pos), _p(vel), _p(species),
                                    _p(self.work), self.work.numel(), _stream(stream),
                                    ctypes.byref(self.handle)))

    def step(self, nsteps: int = 1):
        _check(lib.pasta_sim_step(self.handle, nsteps))

    def energies(self):
        ek, ep, L = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = ctypes.c_int64()
        _check(lib.pasta_sim_energies(self.handle, ctypes.byref(ek), ctypes.byref(ep),
                                      ctypes.byref(L), ctypes.byref(st)))
        return dict(ekin=ek.value, epot=ep.value, L=L.value, step=st.value)

    def forces(self):
        f = torch.empty((self.n, 3), dtype=torch.float64, device=self.pos.device)
        e = torch.empty(self.n, dtype=torch.float64, device=self.pos.device)
        _check(lib.pasta_sim_forces(self.handle, _p(f), _p(e)))
        return f, e

    def pair_counts(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.pasta_sim_pair_counts(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def get_step(self) -> int:
        st = ctypes.c_int64()
        _check(lib.pasta_sim_get_step(self.handle, ctypes.byref(st)))
        return st.value

    def get_state(self, pos=None, vel=None):
        """Copies the current state into `pos` / `vel` (new tensors when not
        given); returns (pos, vel, step)."""
        n = self.pos.shape[0]
        pos = pos if pos is not None else torch.empty((n, 3), dtype=torch.float64,
                                                       device=self.pos.device)
        vel = vel if vel is not None else torch.empty((n, 3), dtype=torch.float64,
                                                       device=self.pos.device)
        st = ctypes.c_int64()
        _check(lib.pasta_sim_get_state(self.handle, _p(pos), _p(vel), ctypes.byref(st)))
        return pos, vel, st.value

    def set_state(self, pos, vel, step: int):
        _check(lib.pasta_sim_set_state(self.handle, _p(pos), _p(vel), step))

    def set_timing(self, on: bool):
        _check(lib.pasta_sim_set_timing(self.handle, int(bool(on))))

    def list_stats(self) -> dict:
        """Neighbour-list counters (all zero unless the list form is on)."""
        b, o, r, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        d = ctypes.c_double()
        _check(lib.pasta_sim_list_stats(self.handle, ctypes.byref(b), ctypes.byref(o),
                                        ctypes.byref(d), ctypes.byref(r), ctypes.byref(c)))
        return dict(builds=b.value, overflows=o.value, max_disp=d.value, rows_used=r.value,
                    rows_capacity=c.value)

    def kernel_times(self):
        ms = (ctypes.c_double * PASTA_KERNEL_CLASSES)()
        nl = (ctypes.c_int64 * PASTA_KERNEL_CLASSES)()
        _check(lib.pasta_sim_kernel_times(self.handle, ms, nl))
        return {pasta_kernel_class_name(k): (ms[k], nl[k]) for k in range(PASTA_KERNEL_CLASSES)}

    def close(self):
        if self.handle:
            lib.pasta_sim_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pasta_sim_create(*args, **kw) -> Sim:
    return Sim(*args, **kw)


# ------------------------------------------------------------------- a5
def pasta_cluster(pos, species, L: float, r_pp: float = 4.5, r_np: float = 3.0, stream=None):
    """Returns dict(label int32 [n], nclusters, hist_A int32 [n+1],
    hist_Z int32 [n+1], nfree) (labels and histograms on the device)."""
    _check_state(pos, species)
    n = pos.shape[0]
    nb = ctypes.c_size_t()
    _check(lib.pasta_cluster_workspace(n, L, r_pp, r_np, ctypes.byref(nb)))
    work = _workspace(nb.value, pos.device)
    label = torch.empty(n, dtype=torch.int32, device=pos.device)
    hA = torch.empty(n + 1, dtype=torch.int32, device=pos.device)
    hZ = torch.empty(n + 1, dtype=torch.int32, device=pos.device)
    K, nf = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.pasta_cluster(n, L, _p(pos), _p(species), r_pp, r_np, _p(label), _p(hA), _p(hZ),
                             ctypes.byref(K), ctypes.byref(nf), _p(work), work.numel(),
                             _stream(stream)))
    return dict(label=label, nclusters=K.value, hist_A=hA, hist_Z=hZ, nfree=nf.value)


# ------------------------------------------------------------------- a6
class Batch:
    """Owner of a pasta_batch handle: nsys systems concatenated in `pos`,
    `vel`, `species` (system s in rows [off_s, off_s + n_s)), advanced
    together by one persistent launch per step (mode 0) or one launch per
    phase (mode 1), replayed from a captured hipGraph."""

    def __init__(self, pos, vel, species, ns, L0s, integs, precision=PASTA_MIXED, mode=0,
                 steps_per_graph=10, step0=0, L_max=None, pot=None, stream=None):
        _check_state(pos, species)
        if vel.shape != pos.shape or vel.dtype != torch.float64 or not vel.is_contiguous():
            raise ValueError("vel must be a contiguous float64 tensor shaped like pos")
        self.nsys = len(ns)
        if sum(ns) != pos.shape[0]:
            raise ValueError("sum of system sizes != number of particles")
        self.pos, self.vel, self.species = pos, vel, species
        self.pot = pot or pasta_potential_paper()
        self.ns = (ctypes.c_int64 * self.nsys)(*ns)
        self.L0 = (ctypes.c_double * self.nsys)(*L0s)
        self.Lmax = (ctypes.c_double * self.nsys)(*(L_max or L0s))
        self.integ = (pasta_integrator * self.nsys)(*[
            pasta_integrator(g.get("dt", 2.0), g.get("xi_dot", 0.0), g.get("T", 1.0),
                             g.get("rescale_every", 0), int(bool(g.get("scale_positions", 0))))
            for g in integs])
        nb = ctypes.c_size_t()
        _check(lib.pasta_batch_workspace(ctypes.byref(self.pot), precision, self.nsys,
                                         self.ns, self.Lmax, ctypes.byref(nb)))
        self.work = _workspace(nb.value, pos.device)
        self.handle = ctypes.c_void_p()
        _check(lib.pasta_batch_create(ctypes.byref(self.pot), precision, self.nsys, self.ns,
                                      self.L0, self.integ, step0, self.Lmax, _p(pos), _p(vel),
                                      _p(species), _p(self.work), self.work.numel(), mode,
                                      steps_per_graph, _stream(stream),
                                      ctypes.byref(self.handle)))

    def step(self, nsteps: int = 1):
        _check(lib.pasta_batch_step(self.handle, nsteps))

    def set_wait_limit(self, polls: int):
        _check(lib.pasta_batch_set_wait_limit(self.handle, polls))

    def energies(self):
        n = self.nsys
        ek, ep, L = (ctypes.c_double * n)(), (ctypes.c_double * n)(), (ctypes.c_double * n)()
        st = ctypes.c_int64()
        _check(lib.pasta_batch_energies(self.handle, ek, ep, L, ctypes.byref(st)))
        return dict(ekin=list(ek), epot=list(ep), L=list(L), step=st.value)

    def forces(self):
        N = self.pos.shape[0]
        f = torch.empty((N, 3), dtype=torch.float64, device=self.pos.device)
        e = torch.empty(N, dtype=torch.float64, device=self.pos.device)
        _check(lib.pasta_batch_forces(self.handle, _p(f), _p(e)))
        return f, e

    def pair_counts(self):
        n = self.nsys
        a, b = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
        _check(lib.pasta_batch_pair_counts(self.handle, a, b))
        return list(a), list(b)

    def info(self):
        g, m = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.pasta_batch_info(self.handle, ctypes.byref(g), ctypes.byref(m)))
        return dict(grid=g.value, mode=m.value)

    def close(self):
        if self.handle:
            lib.pasta_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pasta_batch_create(*args, **kw) -> Batch:
    return Batch(*args, **kw)
