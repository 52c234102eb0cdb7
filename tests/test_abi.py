"""The C-ABI library loads on the CPU and exports every symbol of include/bfc.h."""
import os
import re
import ctypes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bfc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:bf_status|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_four_path_calls():
    names = declared_functions()
    for n in ("build_candidates", "filter_pairs", "eval_barrier", "assemble_grad_hess"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2510_10256_amd as bfc
    so = os.path.join(ROOT, "paper_2510_10256_amd", "libbfc.so")
    assert os.path.exists(so), "build the library first"
    L = ctypes.CDLL(so)
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(declared_functions()) == set(bfc.EXPORTED)


def test_argument_errors_are_reported_without_gpu():
    import paper_2510_10256_amd as bfc
    L = bfc.lib()
    rc = L.bf_scene_create(None, None, 1, 1, None, None)
    assert rc == 1 and b"null" in L.bf_last_error()
    rc = L.build_candidates(None, None, None, None)
    assert rc == 1
