"""The force entry point without allocation (pasta_forces_noalloc, scratch in
a static device array of the library) against pasta_forces (scratch in a
caller workspace), through the C ABI: the same kernels on the same inputs,
so the same bits.  Two calls in a row, the second with a smaller input, so
the second runs on scratch that still holds the first call's contents; a
size whose workspace exceeds the static array is refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_matches_workspace_form():
    import torch
    from paper_1412_8502_amd import binding as B
    from paper_1412_8502_amd import inputs
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    for prec in (B.PASTA_FP64, B.PASTA_MIXED):
        # each input is smaller than the one before (the headline size first)
        for (N, yp, dens, seed) in ((51200, 0.2, 0.08, 1001), (20000, 0.3, 0.06, 11),
                                    (2500, 0.4, 0.04, 12)):
            print("noalloc prec", prec, "N", N, flush=True)
            st = inputs.make_state(N, yp, dens, 1.0, seed)
            pos = torch.tensor(st["pos"], device=dev)
            sp = torch.tensor(st["species"], device=dev)
            ref_f, ref_e = B.pasta_forces(pos, sp, st["L"], precision=prec)
            f = torch.full((N, 3), float("nan"), dtype=torch.float64, device=dev)
            e = torch.full((N,), float("nan"), dtype=torch.float64, device=dev)
            B.pasta_forces_noalloc(pos, sp, st["L"], f, e, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(f, ref_f) and torch.equal(e, ref_e)
            # forces only (no energy output)
            f2 = torch.zeros((N, 3), dtype=torch.float64, device=dev)
            B.pasta_forces_noalloc(pos, sp, st["L"], f2, None, precision=prec)
            torch.cuda.synchronize()
            assert torch.equal(f2, ref_f)
    # beyond the static scratch: refused before any launch, outputs untouched
    N = 2_000_000
    pos = torch.zeros((N, 3), dtype=torch.float64, device=dev)
    sp = torch.zeros(N, dtype=torch.uint8, device=dev)
    f = torch.full((N, 3), 7.0, dtype=torch.float64, device=dev)
    with pytest.raises(B.PastaError) as ex:
        B.pasta_forces_noalloc(pos, sp, 300.0, f, None)
    assert ex.value.code == -3
    assert bool((f == 7.0).all())
