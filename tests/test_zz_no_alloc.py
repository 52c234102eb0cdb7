"""The allocation-free entry point (eval_energy_noalloc) against eval_energy:
the same energies, bitwise, on two calls in a row (the second on a smaller
candidate list), through the C ABI."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


@requires_gpu
def test_noalloc_energy_equals_eval_energy_twice():
    import paper_2510_10256_amd as bfc
    dev = torch.device("cuda:0")
    # larger input first, then a smaller one: the static partials keep the
    # first call's values, which the second must not pick up (both inputs,
    # and the trial point at alpha = 0.01, have no infeasible pair: the
    # energies are finite)
    for sc in (synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0),
               synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80)):
        print(f"[noalloc] {sc.name} V={sc.n_verts}", flush=True)
        p = synth.search_direction(sc)
        cs = bfc.ContactScene(sc, device=dev)
        x = cs._as_x(sc.x)
        pt = torch.tensor(p, dtype=torch.float64, device=dev)
        cs.run(x)
        cs.fit_swept(x, pt)
        alpha = torch.full((1,), 0.01, dtype=torch.float64, device=dev)
        for args in ((x,), (x, pt, alpha)):
            ref = cs.eval_energy(*args).clone()
            got = cs.eval_energy_noalloc(*args).clone()
            torch.cuda.synchronize()
            assert got.item() == ref.item() and np.isfinite(ref.item()) and ref.item() > 0.0, (sc.name, got, ref)
        cs.close()
