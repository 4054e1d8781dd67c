"""C-ABI boundary checks that need no GPU: the library loads, exports every entry
point include/tomo.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tomo.h")

tomo = pytest.importorskip("paper_2206_09151_amd.tomo")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tomo_[a-z_]+)\s*\(", text)))


def test_header_and_library_agree():
    declared = _declared_functions()
    assert len(declared) >= 12
    lib = tomo.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(tomo.EXPORTED) == declared


def test_status_strings():
    lib = tomo.lib()
    for st in range(6):
        assert lib.tomo_status_string(st)
    assert b"domain" in lib.tomo_status_string(tomo.EDOMAIN) or b"<= 0" in lib.tomo_status_string(tomo.EDOMAIN)


def _params(**kw):
    base = dict(n_vox=32, n_angles=4, voxel_size=1e-6, wavelength=1e-10, sigma=0.0, epsilon=1e-3)
    base.update(kw)
    return tomo.Params(**base)


def test_workspace_bytes_counts_stacks():
    p = _params(angle_batch=3)
    ws = tomo.workspace_bytes(p)
    stack = 3 * 32 * 32 * 32 * 4
    assert ws > stack
    assert tomo.workspace_bytes(_params(n_vox=1)) == 0


def _plan_status(p, dirs=None, dist=None):
    lib = tomo.lib()
    d = np.ascontiguousarray(dirs if dirs is not None else [[0.0, 0.0, 1.0]] * p.n_angles, dtype=np.float64)
    r = np.ascontiguousarray(dist if dist is not None else np.zeros(p.n_angles), dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    out = ctypes.c_void_p()
    c = p.to_c()
    st = lib.tomo_plan(ctypes.byref(c), d.ctypes.data_as(dp), None, r.ctypes.data_as(dp), None,
                       ctypes.byref(out))
    return st, lib.tomo_plan_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(n_vox=1), "n_vox"),
    (dict(voxel_size=0.0), "voxel_size"),
    (dict(wavelength=-1.0), "wavelength"),
    (dict(epsilon=0.0), "epsilon"),
    (dict(sigma=float("nan")), "sigma"),
    (dict(ewald=2), "ewald"),
    (dict(tune=6), "tune"),
    (dict(weight_mode=7), "weight_mode"),
    (dict(n_planes=100), "n_planes"),
])
def test_plan_rejects_bad_params(kw, msg):
    st, err = _plan_status(_params(**kw))
    assert st == tomo.EINVAL
    assert msg in err


def test_plan_rejects_non_unit_direction():
    st, err = _plan_status(_params(n_angles=2), dirs=[[0, 0, 1.0], [0, 0, 1.001]])
    assert st == tomo.EINVAL and "unit" in err


def test_plan_rejects_ramp_axis_off_axis_direction():
    d = np.array([[0.0, 0.6, 0.8], [0.0, 0.0, 1.0]])
    st, err = _plan_status(_params(n_angles=2), dirs=d)
    assert st == tomo.EINVAL and "y axis" in err


@pytest.mark.parametrize("m", [14, 98, 112, 264, 7 * 32])
def test_plan_refuses_detector_sizes_outside_the_contract(m):
    """Supported: every M = 2^a 3^b 5^c in [16, 256]; others are refused before any device work."""
    st, err = _plan_status(_params(n_pix=m))
    assert st == tomo.EUNSUPPORTED and "n_pix" in err


def test_plan_refuses_bad_plane_dtype():
    st, err = _plan_status(_params(plane_dtype=7))
    assert st == tomo.EINVAL and "plane_dtype" in err


def test_workspace_halves_with_16bit_planes():
    p32 = tomo.workspace_bytes(_params(angle_batch=4))
    p16 = tomo.workspace_bytes(_params(angle_batch=4, plane_dtype=tomo.BF16))
    assert p32 - p16 == 4 * 32 * 32 * 32 * 2


def test_plan_workspace_limit_gives_enomem():
    st, err = _plan_status(_params(max_workspace_bytes=1024))
    assert st == tomo.ENOMEM and "max_workspace_bytes" in err


def test_null_plan_calls_are_rejected():
    lib = tomo.lib()
    assert lib.tomo_reconstruct(None, None, None, None) == tomo.EINVAL
    assert lib.tomo_reconstruct_async(None, None, None, None) == tomo.EINVAL
    assert lib.tomo_grid(None, None, 0, 1, None, None) == tomo.EINVAL
    assert lib.tomo_backpropagate(None, None, 0, 1, None, None) == tomo.EINVAL
    assert lib.tomo_destroy(None) == tomo.OK
    assert lib.tomo_batch_capacity(None) == 0


def test_fourier_params_checked():
    st, err = _plan_status(_params(fourier=3))
    assert st == tomo.EINVAL and "fourier" in err
    st, err = _plan_status(_params(n_vox=44, n_pix=48, fourier=1))
    assert st == tomo.EUNSUPPORTED and "n_vox" in err
    assert tomo.workspace_bytes(_params(fourier=1)) > tomo.workspace_bytes(_params())
    assert tomo.workspace_bytes(_params(fourier=2)) > tomo.workspace_bytes(_params())


def test_timing_kinds_match_header():
    text = open(HEADER).read()
    m = re.search(r"#define\s+TOMO_TIMING_KINDS\s+(\d+)", text)
    assert m and int(m.group(1)) == len(tomo.KERNEL_KINDS)


def test_null_plan_fourier_call_is_rejected():
    assert tomo.lib().tomo_fourier_reconstruct(None, None, 11, 0.0, None, None) == tomo.EINVAL
    assert tomo.lib().tomo_fourier_reconstruct_async(None, None, 11, 0.0, None, None) == tomo.EINVAL
    assert tomo.lib().tomo_fourier_entries(None) == 0


def test_network_header_and_library_agree():
    text = open(os.path.join(ROOT, "include", "tomo_unet.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = sorted(set(re.findall(r"\b(tomo_unet_[a-z_]+)\s*\(", text)))
    from paper_2206_09151_amd import unet
    assert declared == sorted(unet.EXPORTED)
    lib = tomo.lib()
    for name in declared:
        assert hasattr(lib, name), name
    from oracle import unet as ounet
    assert unet.param_count() == ounet.param_count()


def test_network_rejects_bad_sizes():
    from paper_2206_09151_amd import unet
    for n in (6, 4, 260):
        with pytest.raises(tomo.TomoError) as ei:
            unet.Net(n)
        assert ei.value.status == tomo.EINVAL and "multiple of 4" in str(ei.value)
