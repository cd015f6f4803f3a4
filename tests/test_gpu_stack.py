"""GPU tests of the focal stack through the C ABI.

Every depth of a stack is compared with the float64 oracle's focal stack (each depth reconstructed
with the FrT size shared by the stack) and with a plan at the same depth whose FrT size is forced to
the shared one (the same method through the chained operator passes).
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_13474_amd import nufds as N  # noqa: E402

LAM = 0.5e-6
TOL = {"c128": 1e-10, "c64": 1e-4}
# a depth of the stack against a plan with the same FrT size: the same arithmetic up to the
# rounding of the chain (the plan multiplies the chirp inside its combined pass)
TOL_PLAN = {"c128": 1e-12, "c64": 1e-5}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    N.load()
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _holo(seed, nx, ny, fov, prec, n_points=12):
    dp = synth.fov_pitch(LAM, fov)
    pc = synth.draw_points(seed, n_points, nx, ny, dp, LAM, 1.0e-3, 2.0e-3)
    H = synth.point_hologram(pc, nx, ny, dp, LAM)
    dt = np.complex64 if prec == "c64" else np.complex128
    return dp, H, torch.from_numpy(H.astype(dt)).cuda()


def _rel(a, b):
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_stack_matches_oracle(prec):
    say(f"stack vs oracle {prec}")
    n = 256
    dp, H, Ht = _holo(601, n, n, 90.0, prec)
    zs = [1.6e-3, 1.0e-3, 2.2e-3]
    st = N.Stack(LAM, dp, n, n, zs, precision=prec)
    outs = st(Ht)
    torch.cuda.synchronize()
    refs = O.focal_stack(H, LAM, dp, zs)
    for z, o, r in zip(zs, outs, refs):
        err = O.rel_l2(o.cpu().numpy().astype(np.complex128), r)
        say(f"  z {z:.2e}: rel L2 {err:.3e}")
        assert err <= TOL[prec]
    # every depth uses the size of the nearest one
    sizes = {(i["mx"], i["my"]) for i in st.infos}
    b = O.plan_band(n, n, LAM, dp, 1.0e-3)
    assert sizes == {(b.mx, b.my)}
    st.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_stack_one_pass_row_transforms_match_oracle(prec):
    """A 3888 x 32 hologram at 120 deg whose shared FrT rows are 6400 long, under a 4096-element tile:
    complex64 runs the stack's x transforms in one pass each, the per-depth one multiplying its chirp
    on load from the factored form (c_j a_j^t b_t); complex128 takes the four-step passes."""
    say(f"stack one-pass rows {prec}")
    nx, ny = 3888, 32
    dp, H, Ht = _holo(603, nx, ny, 120.0, prec, n_points=6)
    zs = [2.5e-3, 3.1e-3]
    os.environ["NUFDS_MAX_TILE_ELEMS"] = "4096"
    try:
        st = N.Stack(LAM, dp, nx, ny, zs, precision=prec)
    finally:
        os.environ.pop("NUFDS_MAX_TILE_ELEMS", None)
    assert {i["mx"] for i in st.infos} == {6400}
    outs = st(Ht)
    torch.cuda.synchronize()
    refs = O.focal_stack(H, LAM, dp, zs)
    for z, o, r in zip(zs, outs, refs):
        err = O.rel_l2(o.cpu().numpy().astype(np.complex128), r)
        say(f"  z {z:.2e}: rel L2 {err:.3e}")
        assert err <= TOL[prec]
    st.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_stack_depth_equals_plan_with_shared_size(prec):
    say(f"stack vs forced-size plans {prec}")
    n = 384
    dp, H, Ht = _holo(602, n, n, 120.0, prec)
    zs = [1.2e-3, 2.0e-3]
    st = N.Stack(LAM, dp, n, n, zs, precision=prec)
    outs = st(Ht)
    again = st(Ht)
    torch.cuda.synchronize()
    for a, b in zip(outs, again):
        assert torch.equal(a, b)                      # run to run
    for z, o, info in zip(zs, outs, st.infos):
        plan = N.Plan(LAM, dp, n, n, z, precision=prec, frt_size=(info["mx"], info["my"]))
        ref = plan(Ht)
        torch.cuda.synchronize()
        err = _rel(o, ref)
        say(f"  z {z:.2e}: rel to plan {err:.3e}")
        assert err <= TOL_PLAN[prec]
        for k in ("sx", "sy", "mx", "my", "kcx", "kcy", "fcx0", "fcxn"):
            assert info[k] == plan.info[k]
        assert info["dfx"] == plan.info["dfx"]
        plan.close()
    st.close()


@pytest.mark.parametrize("flags", [N.FLAG_CONVERGING, N.FLAG_NO_STRETCH | N.FLAG_NO_REMAP])
def test_stack_flags_match_oracle(flags):
    say(f"stack flags {flags}")
    n = 192
    dp, H, Ht = _holo(603, n, n, 60.0, "c128")
    zs = [1.0e-3, 1.5e-3]
    st = N.Stack(LAM, dp, n, n, zs, precision="c128", flags=flags)
    outs = st(Ht)
    torch.cuda.synchronize()
    refs = O.focal_stack(H, LAM, dp, zs, flags=flags)
    for o, r in zip(outs, refs):
        assert O.rel_l2(o.cpu().numpy(), r) <= TOL["c128"]
    st.close()


def test_stack_rectangular_hologram_and_one_depth():
    say("stack rectangular")
    nx, ny = 320, 256
    dp, H, Ht = _holo(604, nx, ny, 90.0, "c128")
    for zs in ([1.4e-3, 1.1e-3], [1.3e-3]):
        st = N.Stack(LAM, dp, nx, ny, zs, precision="c128")
        outs = st(Ht)
        torch.cuda.synchronize()
        refs = O.focal_stack(H, LAM, dp, zs)
        for o, r in zip(outs, refs):
            assert tuple(o.shape) == (ny, nx)
            assert O.rel_l2(o.cpu().numpy(), r) <= TOL["c128"]
        st.close()


def test_stack_rejects_bad_outputs():
    say("stack output checks")
    n = 128
    dp, H, Ht = _holo(605, n, n, 60.0, "c64")
    st = N.Stack(LAM, dp, n, n, [1.0e-3, 1.2e-3], precision="c64")
    lib = N.load()
    import ctypes
    o = torch.empty((n, n), dtype=torch.complex64, device="cuda")
    same = (ctypes.c_void_p * 2)(o.data_ptr(), o.data_ptr())
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.nufds_stack_execute(st._h, ctypes.c_void_p(Ht.data_ptr()), same, s) == N.ERR_INVALID_ARG
    holo = (ctypes.c_void_p * 2)(o.data_ptr(), Ht.data_ptr())
    assert lib.nufds_stack_execute(st._h, ctypes.c_void_p(Ht.data_ptr()), holo, s) == N.ERR_INVALID_ARG
    info = N.PlanInfo()
    assert lib.nufds_stack_info(st._h, 2, ctypes.byref(info)) == N.ERR_INVALID_ARG
    st.close()
