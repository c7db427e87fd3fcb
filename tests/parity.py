"""Parity measures and tolerances shared by the GPU tests: the HIP library
against the FP64 oracle on identical input bits.

Forces, for precision p (0 = FP64, 1 = mixed):
  normwise      ||F - F_o||_2 / ||F_o||_2                          <= TOL_F[p]
  per particle  max_i ||F_i - F_o,i|| / max(||F_o,i||, F_rms)       <= TOL_FP[p]
                (F_rms: root mean square of ||F_o,i|| over the compared
                particles, so that a particle whose force nearly cancels is
                measured against the typical force, not against zero)
Energy shares E_i (each pair's energy split evenly between its members):
the same two measures with |.|, TOL_E[p] and TOL_EP[p].

The normwise gates are the ones stated for the method; the per-particle
gates bound every particle, so a large error on a few ordinary particles
cannot hide behind the few close pairs of a random start that dominate
||F_o||.
"""
import numpy as np

TOL_F = {0: 1e-12, 1: 1e-5}
TOL_E = {0: 1e-12, 1: 1e-6}
# per particle: the largest values measured over every GPU parity case are
# about 2.3e-15 (FP64) and 2.0e-6 (mixed, forces) / 1.0e-6 (mixed, energies)
TOL_FP = {0: 1e-12, 1: 1e-5}
TOL_EP = {0: 1e-12, 1: 1e-5}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def per_particle(a, b):
    """max_i |a_i - b_i| / max(|b_i|, rms_i |b_i|), rows as vectors."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    if a.shape[0] == 0:
        return 0.0
    if a.ndim == 1:
        d, m = np.abs(a - b), np.abs(b)
    else:
        d, m = np.linalg.norm(a - b, axis=1), np.linalg.norm(b, axis=1)
    rms = np.sqrt(np.mean(m * m))
    den = np.maximum(m, rms)
    den[den == 0] = 1.0
    return float((d / den).max())


def measure(f, of, e=None, oe=None):
    out = dict(f_norm=rel(f, of), f_pp=per_particle(f, of))
    if e is not None:
        out.update(e_norm=rel(e, oe), e_pp=per_particle(e, oe))
    return out


def check(f, of, prec, e=None, oe=None, what="", say=None):
    """Asserts the normwise and per-particle gates of precision `prec` for
    forces (and energy shares when given); returns the measures."""
    m = measure(f, of, e, oe)
    msg = (f"  parity {what} prec {prec}: F norm {m['f_norm']:.2e} per-particle "
           f"{m['f_pp']:.2e}")
    if e is not None:
        msg += f"; E norm {m['e_norm']:.2e} per-particle {m['e_pp']:.2e}"
    (say or print)(msg)
    assert m["f_norm"] <= TOL_F[prec], (what, m)
    assert m["f_pp"] <= TOL_FP[prec], (what, m)
    if e is not None:
        assert m["e_norm"] <= TOL_E[prec], (what, m)
        assert m["e_pp"] <= TOL_EP[prec], (what, m)
    return m
