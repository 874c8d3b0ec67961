"""Host-side memory plan of the library (gfcc_plan_memory; no GPU needed).

The C60-shaped 120/600/3000 system must fit one 288 GB MI355X: what a BF16-IR solve
holds (the borrowed t2, the FP64 and BF16 operands, a window of 8 slots at restart 30)
stays within 250 GB, and the build's peak (L and t2 resident, FP64 operands, fixed
temporaries and the smallest chunk) within the 288 GB of HBM."""
import pytest

from paper_2010_04768_amd import gfcc

GB = 1e9


def test_plan_c60_shape_fits_one_gpu():
    p = gfcc.plan_memory(120, 600, 3000, precision="bf16", restart=30, window=8)
    assert p["total"] <= 250 * GB, p["total"] / GB
    assert p["build_peak"] <= 250 * GB, p["build_peak"] / GB
    # the ring matrix [Wovvo | Wovov] is the only o^2 v^2 operand the context keeps (FP64)
    assert p["ring"] == pytest.approx(2 * (120 * 600) ** 2 * 8)
    assert p["context_fp64"] - p["ring"] < 0.5 * p["ring"]
    # t2 is the caller's (borrowed), not part of the context
    assert p["input_t2"] == pytest.approx(120 ** 2 * 600 ** 2 * 8)


def test_plan_scales_with_window_and_precision():
    a = gfcc.plan_memory(40, 200, 800, precision="bf16", window=8)
    b = gfcc.plan_memory(40, 200, 800, precision="bf16", window=16)
    assert b["total"] - a["total"] == pytest.approx(8 * a["per_slot"] + (b["sigma_workspace"] - a["sigma_workspace"]))
    f = gfcc.plan_memory(40, 200, 800, precision="fp32", window=8)
    d = gfcc.plan_memory(40, 200, 800, precision="fp64", window=8)
    assert f["context_lowp"] == pytest.approx(2 * a["context_lowp"]) and d["context_lowp"] == 0.0
    g = gfcc.plan_memory(40, 200, 800, precision="bf16", window=8, flexible=True)
    assert g["per_slot"] > a["per_slot"]


def test_plan_rejects_bad_arguments():
    with pytest.raises(gfcc.GfccError):
        gfcc.plan_memory(0, 200, 800)


def test_device_generator_follows_the_host_recipe():
    """synth.make_system_device (used for the 120/600/3000 system, whose arrays are formed on the
    GPU) draws the same numbers as make_system; on the CPU device, in small blocks, every array
    agrees with the host recipe to rounding."""
    torch = pytest.importorskip("torch")
    import numpy as np
    from synth import make_system, make_system_device
    s = make_system(5, 11, 17, 321)
    d = make_system_device(5, 11, 17, 321, "cpu", chunk_bytes=3000)
    assert np.array_equal(d["eps"].numpy(), s.eps)
    assert np.array_equal(d["L"].numpy(), s.L)
    assert np.array_equal(d["t1"].numpy(), s.t1)
    t2 = d["t2"].numpy()
    assert np.abs(t2 - s.t2).max() <= 1e-14 * np.abs(s.t2).max()
