"""Host-side checks of the C ABI: the library loads without a GPU, exports
every function include/gsp.h declares, and rejects bad arguments before
touching the device.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsp_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2410_08743_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        pytest.skip("libgsp.so is not built")
    return N.lib()


def test_header_declarations_are_all_exported(lib):
    from paper_2410_08743_amd import _native as N
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), f"{name} declared in gsp.h but not exported"
    assert sorted(N.EXPORTS) == names


def test_version_and_status_strings(lib):
    assert lib.gsp_version() == 1
    assert lib.gsp_status_string(0) == b"ok"
    assert b"capacity" in lib.gsp_status_string(2)


def test_workspace_size_validates_views(lib):
    from paper_2410_08743_amd import _native as N
    from paper_2410_08743_amd.synthetic import Camera
    sz = ctypes.c_size_t()
    good = N.view_array([Camera(100, 80, 90.0, 90.0, 50.0, 40.0)])
    assert lib.gsp_workspace_size(1000, 3, 1, good, 10000, ctypes.byref(sz)) == N.GSP_OK
    small = sz.value
    assert lib.gsp_workspace_size(1000, 3, 1, good, 20000, ctypes.byref(sz)) == N.GSP_OK
    assert sz.value > small
    bad_roi = N.view_array([Camera(100, 80, 90.0, 90.0, 50.0, 40.0, roi=(8, 0, 16, 16))])
    assert lib.gsp_workspace_size(1000, 3, 1, bad_roi, 100, ctypes.byref(sz)) == N.GSP_EINVAL
    assert b"multiple of 16" in lib.gsp_last_error()
    outside = N.view_array([Camera(100, 80, 90.0, 90.0, 50.0, 40.0, roi=(96, 0, 16, 16))])
    assert lib.gsp_workspace_size(1000, 3, 1, outside, 100, ctypes.byref(sz)) == N.GSP_EINVAL
    assert lib.gsp_workspace_size(1000, 4, 1, good, 100, ctypes.byref(sz)) == N.GSP_EINVAL
    assert lib.gsp_workspace_size(-1, 0, 1, good, 100, ctypes.byref(sz)) == N.GSP_EINVAL
    assert lib.gsp_workspace_size(10, 0, 0, good, 100, ctypes.byref(sz)) == N.GSP_EINVAL
    many = N.view_array([Camera(32, 32, 30.0, 30.0, 16.0, 16.0)] * 33)
    assert lib.gsp_workspace_size(10, 0, 33, many, 100, ctypes.byref(sz)) == N.GSP_EINVAL


def test_calls_reject_null_context(lib):
    from paper_2410_08743_amd import _native as N
    assert lib.gsp_render_fwd(None, None, 1, None, None, None, None, None, 0, 0, None) == N.GSP_EINVAL
    assert lib.gsp_loss_l1(None, 1, None, None, None, None, None, None, None) == N.GSP_EINVAL
    assert lib.gsp_pose_adam(None, 1, None, None, None, None, None, None, None, None) == N.GSP_EINVAL
    assert lib.gsp_loss_rgb(None, 1, None, None, None, None, None, 0.2, None, 0, None) == N.GSP_EINVAL
    assert lib.gsp_gaussian_adam(None, 1, 0, None, None, None, None, 1, None, None, None, None,
                                 None, None, None) == N.GSP_EINVAL
    assert lib.gsp_create(0, None) == N.GSP_EINVAL


def test_scratch_sizes_of_the_joint_calls(lib):
    from paper_2410_08743_amd import _native as N
    from paper_2410_08743_amd.synthetic import Camera
    one = N.view_array([Camera(100, 37, 90.0, 90.0, 50.0, 18.0)])
    # two 64 x 16 tiles across, three down; per-tile sums of 3 channels + 9 floats per pixel
    tiles = 2 * 3
    expect = ((3 * tiles * 16 + 255) // 256) * 256 + 9 * 100 * 37 * 4
    assert lib.gsp_loss_rgb_scratch_bytes(1, one) == expect
    two = N.view_array([Camera(100, 37, 90.0, 90.0, 50.0, 18.0)] * 2)
    assert lib.gsp_loss_rgb_scratch_bytes(2, two) == ((3 * 2 * tiles * 16 + 255) // 256) * 256 + 2 * 9 * 100 * 37 * 4
    # L_An partial sums: one per 256-item block holding log-scale items (items 3n .. 4n)
    assert lib.gsp_gaussian_adam_scratch_bytes(1000) == 8 * ((4000 - 1) // 256 - 3000 // 256 + 1)
    assert lib.gsp_gaussian_adam_scratch_bytes(0) == 8


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2410_08743_amd import _native as N
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(N, "_lib", None)
    with pytest.raises(N.NativeLibraryMissing):
        N.lib()


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2410_08743_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "gso_" not in text and "liboracle" not in text, f
