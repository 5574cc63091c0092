"""The C ABI loads, exports what include/bst.h declares, and rejects bad
arguments on the host before any device work. CPU only (no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1704_08364_amd as P
from paper_1704_08364_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "bst.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bst_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = _declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(binding.SIGNATURES), "binding signatures out of sync with bst.h"


def _params(**kw):
    p, keep = P.make_params(kw.pop("n", 256), kw.pop("V", 256), kw.pop("N", None), **kw)
    return p, keep


def _validate(p):
    return P.lib().bst_validate(C.byref(p))


def test_defaults_validate():
    p, _ = _params()
    assert _validate(p) == 0
    assert p.pad_radial == 2 and p.pad_cart == 2 and p.filter == 1 and p.taper == 0


@pytest.mark.parametrize("field,value,code", [
    ("n_det", 100, 2), ("n_det", 8, 2), ("n_det", 8192, 2), ("n_out", 128, 2),
    ("n_angles", 1, 2), ("n_angles", 20000, 2),
    ("pad_radial", 3, 4), ("pad_cart", 8, 4), ("filter", 2, 4), ("taper", 7, 4),
    ("max_batch", 0, 9), ("device", -1, 4), ("interp", 2, 4), ("interp", -1, 4),
    ("gather_slices", 3, 4), ("gather_slices", -2, 4), ("gather_slices", 1026, 4),
    ("dtype", 2, 4), ("dtype", -1, 4),
])
def test_validation_codes(field, value, code):
    p, _ = _params()
    setattr(p, field, value)
    assert _validate(p) == code


def test_transform_length_limit():
    p, _ = _params(n=4096, V=64, pad_radial=2, pad_cart=2)  # M = G = 8192: the largest
    assert _validate(p) == 0
    p.pad_radial = 4
    assert _validate(p) == 2
    p.pad_radial, p.pad_cart = 2, 4
    assert _validate(p) == 2


def test_kaiser_beta_checked():
    p, _ = _params(taper="kaiser", taper_beta=-1.0)
    assert _validate(p) == 4
    p.taper_beta = float("nan")
    assert _validate(p) == 4
    p.taper_beta = 6.0
    assert _validate(p) == 0


@pytest.mark.parametrize("angles,code", [
    ([0.0, 0.5, 0.5, 1.0], 3),
    ([0.0, 0.5, 1.0, 3.2], 3),
    ([-0.1, 0.5, 1.0, 2.0], 3),
    ([0.0, float("nan"), 1.0, 2.0], 3),
    ([0.0, 0.5, 1.0, 2.0], 0),
])
def test_angle_validation(angles, code):
    p, keep = _params(n=64, V=4, angles=angles)
    assert _validate(p) == code


def test_null_arguments():
    L = P.lib()
    assert L.bst_validate(None) == 1
    size = C.c_size_t()
    assert L.bst_query_workspace(None, 1, C.byref(size)) == 1
    p, _ = _params()
    assert L.bst_query_workspace(C.byref(p), 1, None) == 1
    assert L.bst_plan(C.byref(p), None) == 1
    assert L.bst_backproject(None, None, None, 1, None, 0, None) == 1
    assert L.bst_backproject_bruteforce(None, None, None, 1, None) == 1
    assert L.bst_project(None, None, None, 1, None, 0, None) == 1
    assert L.bst_destroy(None) == 0


def test_workspace_size_is_exact_and_monotone():
    p, _ = _params(n=2048, V=2048, max_batch=64)
    sizes = [P.query_workspace(p, b) for b in (0, 1, 2, 7, 64)]
    assert sizes[0] == 0
    assert all(a < b for a, b in zip(sizes, sizes[1:]))
    # polar spectra per group of 2 slices: ceil(V/2) rows of ceil((M/2+2)/4)
    # tiles of 2 angles x 4 samples x 2 slices (128 bytes); + dc [V] f32 + grid
    # [N][G/2] c64 per slice, 256-byte aligned blocks
    group = 1024 * 513 * 128
    per = 2048 * 4 + 2048 * 2048 * 8
    assert abs(sizes[1] - (group + per)) < 3 * 256
    assert abs(sizes[2] - (group + 2 * per)) < 3 * 256
    assert abs(sizes[3] - (4 * group + 7 * per)) < 3 * 256
    assert abs(sizes[4] - (32 * group + 64 * per)) < 3 * 256
    with pytest.raises(P.BstError):
        P.query_workspace(p, 65)
    with pytest.raises(P.BstError):
        P.query_workspace(p, -1)


def test_status_strings():
    L = P.lib()
    for code in range(11):
        assert L.bst_status_string(code)
    assert b"unknown" in L.bst_status_string(99)


def test_plan_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p, _ = _params()
    h = C.c_void_p(1234)
    assert P.lib().bst_plan(C.byref(p), C.byref(h)) == 7
    assert h.value is None
    with pytest.raises(P.BstError):
        P.Plan(256, 256)


def test_adjoint_workspace_covers_both_directions():
    p, _ = _params(n=1024, V=1024, max_batch=17)
    plain = P.query_workspace(p, 8)
    p.adjoint = 1
    both = P.query_workspace(p, 8)
    # projector: grid [N][G/2] + Cartesian half plane [G/2][G] with 16 slices
    # interleaved for the transposed gather (whole groups of 16) + polar [V][M/2],
    # complex64
    N = V = 1024
    G = M = 2048
    for B in (8, 3, 17):
        p.adjoint = 0
        plain = P.query_workspace(p, B)
        p.adjoint = 1
        both = P.query_workspace(p, B)
        groups = -(-B // 16)
        proj = 8 * (B * N * G // 2 + groups * 16 * G // 2 * G + B * V * M // 2)
        assert both >= plain and abs(both - max(plain, proj)) < 5 * 256


def test_batch_create_validates_before_device_work():
    L = P.lib()
    p, _ = _params()
    h = C.c_void_p()
    n = (C.c_int32 * 3)(256, 512, 100)
    v = (C.c_int32 * 3)(128, 256, 64)
    assert L.bst_batch_create(None, 3, n, v, C.byref(h)) == 1
    assert L.bst_batch_create(C.byref(p), 0, n, v, C.byref(h)) == 9
    assert L.bst_batch_create(C.byref(p), 3, n, v, C.byref(h)) == 2  # 100 is not a power of two
    # per-instance angle counts exclude a shared angle list; FP64 runs one plan at a time
    th = np.arange(256) * (np.pi / 256)
    pa, _keep = _params(angles=th)
    assert L.bst_batch_create(C.byref(pa), 3, n, v, C.byref(h)) == 8
    pf, _ = _params(dtype="f64")
    assert L.bst_batch_create(C.byref(pf), 3, n, v, C.byref(h)) == 8
    assert h.value is None
    assert L.bst_batch_destroy(None) == 0


def test_keys_interpolation_validates_and_sizes_its_rows():
    p, _ = _params(n=2048, V=2048, max_batch=4, taper="keys", interp="keys")
    assert _validate(p) == 0
    # keys rows: one leading slot and four trailing zeros, [V][M/2 + 5], one
    # slice per polar group (linear taps interleave two)
    per = 2048 * (2048 + 5) * 8 + 2048 * 4 + 2048 * 2048 * 8
    assert abs(P.query_workspace(p, 1) - per) < 3 * 256
    assert abs(P.query_workspace(p, 3) - 3 * per) < 4 * 256
    lin, _ = _params(n=2048, V=2048, max_batch=4)
    assert P.query_workspace(p, 4) > P.query_workspace(lin, 4)
    # the projector is the exact transpose of the cubic gather too
    p.adjoint = 1
    assert _validate(p) == 0


def test_adjoint_takes_non_uniform_angles():
    import numpy as np
    p, keep = _params(n=64, V=8, angles=np.linspace(0.1, 3.0, 8))
    assert _validate(p) == 0
    p.adjoint = 1
    assert _validate(p) == 0
    assert P.query_workspace(p, 1) > 0


@pytest.mark.parametrize("kw,code", [
    (dict(filter="none", monopole_width=0.4), 0),
    (dict(filter="none", monopole_width=4 * 2.0 / 256), 0),        # the narrowest: 4 dt
    (dict(filter="none", monopole_width=2.0), 0),
    (dict(filter="ramp", monopole_width=0.4), 4),                   # plain B only
    (dict(filter="none", monopole_width=0.4, adjoint=True), 4),     # no longer the transpose
    (dict(filter="none", monopole_width=3.9 * 2.0 / 256), 4),       # under-resolved
    (dict(filter="none", monopole_width=2.5), 4),
    (dict(filter="none", monopole_width=-0.4), 4),
    (dict(filter="none", monopole_width=float("nan")), 4),
    (dict(filter="none", monopole_width=float("inf")), 4),
])
def test_monopole_validation(kw, code):
    p, _ = _params(n=256, V=128, **kw)
    assert _validate(p) == code


def test_monopole_workspace_adds_the_partial_sums():
    for B in (1, 3, 64):
        plain, _ = _params(n=256, V=128, filter="none", max_batch=B)
        mono, _ = _params(n=256, V=128, filter="none", max_batch=B, monopole_width=0.4)
        a = P.query_workspace(plain, B)
        b = P.query_workspace(mono, B)
        # [B][64] float32 partial sums, rounded to 256 bytes
        assert b - a == -(-B * 64 * 4 // 256) * 256


def test_max_batch_is_the_largest_that_fits():
    # Section 4's bound on the block size Q: sinograms + images + workspace <= budget
    for kw in (dict(), dict(filter="none", monopole_width=0.4), dict(adjoint=True), dict(interp="keys")):
        p, _ = _params(n=256, V=200, max_batch=500, **kw)

        def need(q):
            return q * (200 * 256 + 256 * 256) * 4 + P.query_workspace(p, q)

        for q in (1, 2, 7, 64, 499):
            assert P.query_max_batch(p, need(q)) == q
            assert P.query_max_batch(p, need(q + 1) - 1) == q
        assert P.query_max_batch(p, need(500) * 4) == 500          # capped at max_batch
        assert P.query_max_batch(p, need(1) - 1) == 0


def test_max_batch_codes():
    L = P.lib()
    p, _ = _params(n=256, V=200, max_batch=8)
    q = C.c_int32(-1)
    assert L.bst_query_max_batch(C.byref(p), 0, C.byref(q)) == 6 and q.value == 0   # BST_E_NOMEM
    assert L.bst_query_max_batch(C.byref(p), 1 << 40, None) == 1
    assert L.bst_query_max_batch(None, 1 << 40, C.byref(q)) == 1
    p.n_det = 100
    assert L.bst_query_max_batch(C.byref(p), 1 << 40, C.byref(q)) == 2
    # 288 GB of HBM holds far more than a 2048^2 x 2048-angle batch of 64
    p2, _ = _params(n=2048, V=2048, max_batch=4096)
    assert 64 < P.query_max_batch(p2, 288 * 10**9) < 4096


@pytest.mark.parametrize("kw,code", [
    (dict(angular="tent"), 0),
    (dict(angular="tent", filter="none", adjoint=True), 0),
    (dict(angular="tent", interp="keys", taper="keys"), 4),          # linear radial taps only
    (dict(angular="tent", angles=np.linspace(0, 3.0, 128)), 4),     # uniform angles only
    (dict(angular=2), 4),
    (dict(angular=-1), 4),
    (dict(angular="tent", V=790), 0),                                 # V/pi = 251.5 < G/2 - 1 = 255
    (dict(angular="tent", V=802), 4),                                 # V/pi = 255.3: the disk leaves the grid
])
def test_tent_validation(kw, code):
    kw = dict(kw)
    p, _ = _params(n=256, V=kw.pop("V", 128), **kw)
    assert _validate(p) == code


def test_tent_workspace_adds_the_wide_points():
    # wide points: a^2 + b^2 < (V/pi)^2 over the half-plane columns a >= 0, plus
    # a radius-major copy of the radial samples they read (m <= floor(V/pi) + 1
    # at P_r = P_c), complex64 per slice
    # (8 slices interleaved, whole groups), and the pre-gather's chunk sums:
    # each point's tap range floor(q-h)-1 .. ceil(q+h)+1 in chunks of 32, one
    # complex sum per slice and one weight sum per chunk
    import math
    n, V = 256, 300
    R = V / np.pi
    W, C = 0, 0
    for a in range(int(np.ceil(R))):
        Bc = int(np.floor(np.sqrt(R * R - a * a) - 1e-12))
        W += 2 * Bc + 1
        for b in range(-Bc, Bc + 1):
            if a == 0 and b == 0:
                continue
            rho = math.hypot(a, b)
            phi = math.atan2(b, a)
            q = (phi + math.pi if phi < 0 else phi) * V / math.pi
            h = V / (math.pi * rho)
            lo, hi = math.floor(q - h) - 1, math.ceil(q + h) + 1
            C += -(-(hi - lo + 1) // 32)
    rows = min(int(np.floor(R)) + 2, n)

    def up(x):
        return -(-x // 256) * 256

    for B in (1, 5, 9, 17):
        plain, _ = _params(n=n, V=V, max_batch=B)
        tent, _ = _params(n=n, V=V, max_batch=B, angular="tent")
        extra = P.query_workspace(tent, B) - P.query_workspace(plain, B)
        # values [B][W], the copy for whole groups of 8 slices, chunk sums [B][C], weight sums [C]
        groups = -(-B // 8)
        assert extra == up(B * W * 8) + up(groups * 8 * rows * V * 8) + up(B * C * 8) + up(C * 4)


def test_debug_check_in_the_ordinary_build():
    L = P.lib()
    flags = C.c_uint32(7)
    assert L.bst_debug_check(0, None) == 1
    if os.path.basename(binding.LIB_PATH) == "libbst.so":
        assert L.bst_debug_check(0, C.byref(flags)) == 8 and flags.value == 0


def test_fp64_plans_validate_and_size():
    # the FP64 gradient-check path: n <= 512, uniform angles, linear taps, no monopole
    p, _ = _params(n=256, V=200, dtype="f64", max_batch=3)
    assert _validate(p) == 0
    size = P.query_workspace(p, 3)
    # polar [V][M/2+2] + dc [V] + Cartesian [G][G/2+1] + polar^T [V][M/2+1] (16-byte complex) + origin
    M = G = 512
    expect = 3 * (200 * (M // 2 + 2) * 16 + 200 * 8 + G * (G // 2 + 1) * 16 + 200 * (M // 2 + 1) * 16 + 8)
    assert abs(size - expect) < 6 * 256
    for kw in (dict(n=1024, V=64), dict(n=256, V=64, interp="keys", taper="keys"),
               dict(n=256, V=64, angular="tent"), dict(n=256, V=64, filter="none", monopole_width=0.4),
               dict(n=64, V=4, angles=[0.1, 0.5, 1.0, 2.0])):
        q, _keep = _params(dtype="f64", **kw)
        assert _validate(q) == 8, kw
    L = P.lib()
    assert L.bst_backproject_f64(None, None, None, 1, None, 0, None) == 1
    assert L.bst_project_f64(None, None, None, 1, None, 0, None) == 1
