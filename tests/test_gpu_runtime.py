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


@requires_gpu
def test_threads_per_query_choices_give_the_same_candidates():
    # every choice of threads per broad-phase query (2, 4, 8, 16) finds the
    # same candidate pairs (in another order within a query), and the tuner
    # picks one of them; the per-thread buffers hold the largest choice
    import paper_2510_10256_amd as bfc
    sc = synth.folded_cloth(n=72, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)
    cs = bfc.ContactScene(sc, device="cuda:0")
    x = cs._as_x(sc.x)
    try:
        sets = {}
        for pq in (2, 4, 8, 16):
            print(f"[pq] {sc.name} V={sc.n_verts} pq={pq}", flush=True)
            cs.set_pq(pq)
            st = cs.run(x)
            assert not (st & bfc.binding.BF_S_CAND_OVERFLOW)
            n = int(cs.c_n.item())
            key = (cs.c_t[:n].to(torch.int64) << 62) | (cs.c_i[:n].to(torch.int64) << 31) | cs.c_j[:n].to(torch.int64)
            sets[pq] = np.sort(key.cpu().numpy())
            assert len(np.unique(sets[pq])) == n
        for pq in (2, 8, 16):
            assert np.array_equal(sets[pq], sets[4]), pq
        assert cs.tune(x) in (2, 4, 8, 16)
    finally:
        cs.close()


@requires_gpu
def test_scene_in_a_caller_workspace():
    # bf_scene_create_ws carves the scene from a caller's tensor of
    # bf_workspace_bytes bytes: the step's results are bitwise those of a
    # scene the library allocates; one byte less is refused, and the scene
    # cannot grow
    import ctypes as C
    import paper_2510_10256_amd as bfc
    from paper_2510_10256_amd import binding as B
    sc = synth.folded_cloth(n=48, gaps=(950.0,), l_mid=4000.0, l_conv=2000.0)
    print(f"[workspace] {sc.name} V={sc.n_verts}", flush=True)
    ref = bfc.ContactScene(sc, device="cuda:0")
    x = ref._as_x(sc.x)
    st = ref.run(x)  # grows its buffers until the step fits
    assert not (st & (B.BF_S_CAND_OVERFLOW | B.BF_S_ACT_OVERFLOW | B.BF_S_BSR_OVERFLOW))
    cs = bfc.ContactScene(sc, device="cuda:0", own_workspace=True, cand_cap=ref.cand_cap, act_cap=ref.act_cap,
                          bsr_cap=ref.bsr_cap)
    try:
        cs.step(x)
        assert cs.status(clear=True) == st
        a, b = ref.results(), cs.results()
        assert a["counts"] == b["counts"] and a["E_total"] == b["E_total"]
        for k in ("g", "row_ptr", "col", "val", "E", "G", "Hpsd", "cand", "i", "j", "flags", "d"):
            assert np.array_equal(a[k], b[k]), k
        nbytes = cs.workspace.numel()
        # the same arguments, one byte short
        desc = B.MeshDesc(1, sc.n_verts, sc.n_edges, sc.n_tris, cs._edges.ctypes.data, cs._tris.ctypes.data,
                          cs._ref.ctypes.data)
        prm = B.Params(cs.h, cs.eta, cs.kappa, 0, 0, 11)
        h = C.c_void_p()
        rc = B.lib().bf_scene_create_ws(C.byref(desc), C.byref(prm), cs.cand_cap, cs.act_cap,
                                        cs.workspace.data_ptr(), nbytes - 256, C.c_void_p(cs._stream()),
                                        C.byref(h))
        assert rc == 4 and b"workspace" in B.lib().bf_last_error()
        assert B.lib().bf_scene_reserve(cs.handle, 2 * cs.cand_cap, cs.act_cap) == 5
        assert B.lib().bf_scene_reserve(cs.handle, cs.cand_cap, cs.act_cap) == 0
    finally:
        cs.close()
        ref.close()
