"""The C-ABI library loads and exports every symbol include/cvo.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "cvo.h")
LIB = os.path.join(ROOT, "paper_2012_03683_amd", "libcvo_hip.so")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cvo_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for must in ("cvo_inner_product", "cvo_gradient", "cvo_align", "cvo_metric", "cvo_cosine", "cvo_odometry", "cvo_select_points", "cvo_align_replay",
                 "cvo_inner_product_backward", "cvo_align_batched", "cvo_create", "cvo_destroy"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_python_binding_declares_every_export():
    import paper_2012_03683_amd as cvo
    assert sorted(cvo.EXPORTS) == sorted(n for n in declared() if n not in ("cvo_evaluate_batched",))
    lib = cvo.load_library()
    for name in cvo.EXPORTS:
        assert hasattr(lib, name)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_struct_sizes_match_header_layout():
    import paper_2012_03683_amd as cvo
    # sizes implied by the C declarations on x86-64
    assert ctypes.sizeof(cvo.cvo_cloud) == 24
    assert ctypes.sizeof(cvo.cvo_feature_spec) == 4 + 32 + 32 + 4 + 64 + 64
    assert ctypes.sizeof(cvo.cvo_kernel_params) == 24
    assert ctypes.sizeof(cvo.cvo_align_params) == 9 * 8 + 8 + 16
    assert ctypes.sizeof(cvo.cvo_align_report) == 56
    assert ctypes.sizeof(cvo.cvo_eval) == 8 * 12
    assert ctypes.sizeof(cvo.cvo_tuning) == 48
    assert ctypes.sizeof(cvo.cvo_camera) == 48
    assert ctypes.sizeof(cvo.cvo_timing) == 9 * 8


def test_product_path_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_2012_03683_amd as cvo
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    x = torch.zeros((4, 3))
    with pytest.raises(RuntimeError):
        cvo.cvo_inner_product(x, x, [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], 0.1)
