"""GPU tests of the library's runtime behaviour around the path: the
single-pass scan's bounded wait, and the streams a batch capture leaves in
the scenes."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


@requires_gpu
def test_scan_that_stops_waiting_stays_exact():
    # with a wait bound of zero loads, every work-group of a single-pass scan
    # after the first sums the earlier tiles of the input itself: the step's
    # results are bitwise those of the ordinary scan, and BF_S_SCAN_SLOW is
    # raised (forced from the host: no kernel waits or faults)
    import paper_2510_10256_amd as bfc
    sc = synth.woven_patch()  # 32k vertices, 65k cells: scans of 17 to 64 tiles
    print(f"[scan bound] {sc.name} V={sc.n_verts}", flush=True)
    cs = bfc.ContactScene(sc)
    try:
        st = cs.run(sc.x)
        assert not (st & bfc.binding.BF_S_SCAN_SLOW)
        ref = cs.results()
        bfc.lib().bf_set_scan_poll_limit(0)
        cs.step(cs._as_x(sc.x))
        st = cs.status(clear=True)
        got = cs.results()
    finally:
        bfc.lib().bf_set_scan_poll_limit(1 << 22)
        cs.close()
    assert st & bfc.binding.BF_S_SCAN_SLOW
    for k in ("cand", "i", "j", "ptype", "flags", "code", "E", "G", "Hpsd", "g", "row_ptr", "col", "val"):
        assert np.array_equal(ref[k], got[k]), k
    assert ref["E_total"] == got["E_total"]


@requires_gpu
def test_batch_destroyed_without_a_step_leaves_scenes_usable():
    # the capture records lane streams of the batch in the scenes' calls; the
    # scenes must keep their own stream so that reading their status word and
    # destroying them after the batch is gone is well defined
    import paper_2510_10256_amd as bfc
    scenes = [synth.helix_loop_rod(), synth.woven_patch(n_warp=4, n_weft=4, verts_per_rod=80)]
    print("[batch no step] two scenes", flush=True)
    css = [bfc.ContactScene(s) for s in scenes]
    xs = [cs._as_x(s.x) for cs, s in zip(css, scenes)]
    for cs, x in zip(css, xs):
        cs.run(x)
    b = bfc.Batch(css, xs, lanes=2)
    b.close()
    torch.cuda.synchronize()
    for cs, s, x in zip(css, scenes, xs):
        assert cs.status(clear=True) == 0
        cs.run(x)  # the scene still steps on its own
        assert cs.counts()["n_act"] > 0
        cs.close()
