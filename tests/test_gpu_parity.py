"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar (stated in the tests): FP32 end-to-end BST within relative L2 1e-5 of the
FP64 oracle on the same FP32 input bytes; the polar spectrum stage within 1e-6;
brute force within 1e-5. Sizes span several FFT lengths, odd and ragged
angle counts, every padding combination, both filters, all tapers and both
radial interpolations (linear, Keys cubic), plus
the full 64 x 2048 x 2048 batch in the launch configuration the benchmark
times (two of its slices checked in full against the oracle). The projector
(the exact adjoint) is held to the same 1e-5 against the oracle's transpose,
plus the adjoint identity, determinism and autograd gradient checks.
"""
import math
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import bruteforce as obf
from oracle import bst as obst
from oracle import ramp as oramp
from oracle.geometry import Geometry

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    dt = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a = a.astype(dt)
    b = b.astype(dt)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def assert_parity(got, ref, tol=1e-5, elem=1e-4):
    """The parity bar: relative L2 within tol, and no element further than
    elem * max|ref| from the reference (so a local defect cannot hide in the
    global norm)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = rel_l2(got, ref)
    worst = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert err <= tol, f"rel-L2 {err:.3e} > {tol}"
    assert worst <= elem, f"max |difference| {worst:.3e} of max |ref| > {elem}"
    return err, worst


@pytest.fixture(scope="module")
def P():
    import paper_1704_08364_amd as mod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mod.lib()  # fails loudly when libbst.so is missing
    return mod


def _sinos(B, V, n, seed, kind="mixed"):
    """[B][V][n] float32 on the GPU: ellipse phantoms with noise, plus random slices."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    out = synth.batch_sinograms(B, n, V, seed, device=DEV)
    if kind == "mixed" and B > 1:
        out[B - 1] = torch.randn(V, n, generator=g).to(DEV)
    return out


CASES = [
    # N, V, filter, P_r, P_c, taper
    (16, 10, "ramp", 2, 2, "deapod"),
    (16, 7, "none", 1, 1, "none"),
    (32, 24, "none", 2, 2, "deapod"),
    (32, 33, "ramp", 4, 1, "kaiser"),
    (64, 50, "ramp", 1, 2, "deapod"),
    (64, 33, "none", 2, 1, "deapod"),
    (128, 96, "ramp", 4, 2, "none"),
    (128, 128, "ramp", 2, 4, "deapod"),
    (256, 301, "none", 2, 2, "kaiser"),
    (512, 400, "ramp", 2, 2, "deapod"),
    (1024, 256, "ramp", 2, 2, "deapod"),
]


@pytest.mark.parametrize("N,V,filt,P_r,P_c,taper", CASES)
def test_spectrum_stage(P, N, V, filt, P_r, P_c, taper):
    _say(f"[spectrum] N={N} V={V} {filt} Pr={P_r} Pc={P_c} {taper}")
    B = 3
    plan = P.Plan(N, V, pad_radial=P_r, pad_cart=P_c, filter=filt, taper=taper, max_batch=B)
    sino = _sinos(B, V, N, 1000 + N + V)
    spec, dc = plan.debug_spectrum(sino)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(P_r, P_c, filt, taper if taper != "kaiser" else "kb", 8.0)
    M = P_r * N
    for b in range(B):
        Yh, Y0 = obst.spectrum(sino[b].double().cpu().numpy(), geom, prm)
        got = spec[b].cpu().numpy().astype(np.complex128)
        assert rel_l2(got, Yh[:, :M // 2]) <= 1e-6
        assert rel_l2(dc[b].cpu().numpy(), Y0) <= 1e-6


@pytest.mark.parametrize("N,V,filt,P_r,P_c,taper", CASES)
def test_backproject_matches_oracle(P, N, V, filt, P_r, P_c, taper):
    _say(f"[backproject] N={N} V={V} {filt} Pr={P_r} Pc={P_c} {taper}")
    B = 3
    plan = P.Plan(N, V, pad_radial=P_r, pad_cart=P_c, filter=filt, taper=taper, max_batch=B)
    sino = _sinos(B, V, N, 2000 + N + V)
    img = plan.backproject(sino)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(P_r, P_c, filt, taper if taper != "kaiser" else "kb", 8.0)
    for b in range(B):
        ref = obst.backproject(sino[b].double().cpu().numpy(), geom, prm)
        err, worst = assert_parity(img[b].cpu().numpy(), ref)
        _say(f"   slice {b}: rel-L2 {err:.2e}, max {worst:.2e}")


def test_config1_head_phantom(P):
    """256 angles x 256 bins, 10-ellipse head phantom with 1% noise, both filters."""
    sino, g, _ = synth.config1_sinogram(device=DEV)
    geom = Geometry(256, 256, 256)
    y64 = sino.double().cpu().numpy()
    for filt in ("ramp", "none"):
        _say(f"[config1] {filt}")
        plan = P.Plan(256, 256, filter=filt)
        img = plan.backproject(sino)
        ref = obst.backproject(y64, geom, obst.Params(2, 2, filt))
        assert rel_l2(img.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("interp,pad_cart", [("linear", 2), ("keys", 1)])
def test_full_batch_2048(P, interp, pad_cart):
    """64 slices of 2048 angles x 2048 bins: the batch and plans the benchmark
    times (the default path, and the cubic-tap P_c = 1 path its accuracy leg
    quotes); slices 0 and 63 are compared in full with the oracle, and (once)
    a sample of brute-force pixels of slice 7 with the oracle's B_d."""
    B, N, V = 64, 2048, 2048
    _say(f"[full 2048 {interp} P_c={pad_cart}] generating")
    sino = synth.batch_sinograms(B, N, V, seed=170408366, device=DEV)
    kw = dict(taper="keys", interp="keys") if interp == "keys" else {}
    plan = P.Plan(N, V, max_batch=B, pad_cart=pad_cart, **kw)
    ws = plan.workspace(B)
    img = torch.empty(B, N, N, dtype=torch.float32, device=DEV)
    plan.backproject(sino, out=img, workspace=ws)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(2, pad_cart, **kw)
    for b in (0, B - 1):
        _say(f"[full 2048] oracle slice {b}")
        ref = obst.backproject(sino[b].double().cpu().numpy(), geom, prm)
        err, worst = assert_parity(img[b].cpu().numpy(), ref)
        _say(f"   rel-L2 {err:.2e}, max {worst:.2e}")
    if interp != "linear":
        return
    _say("[full 2048] brute force")
    bf = plan.bruteforce(sino[:8])
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    rows = rng.integers(0, N, 3000)
    cols = rng.integers(0, N, 3000)
    ref = obf.backproject_pixels(sino[7].double().cpu().numpy(), geom, rows, cols)
    got = bf[7].cpu().numpy()[rows, cols]
    assert rel_l2(got, ref) <= 1e-5


# Every slices-per-block value the batch tuner may pick (and the smallest and
# largest others), each checked in full on slices of the benchmark's plan: the
# chunking of slices over blocks must not change a result.
@pytest.mark.parametrize("spb", [2, 4, 8, 16, 32, 64])
def test_gather_slices_per_block_variants(P, spb):
    N, V, B = 2048, 2048, 10
    sino = synth.batch_sinograms(B, N, V, seed=170408366, device=DEV)
    plan = P.Plan(N, V, max_batch=B, gather_slices=spb)
    img = plan.backproject(sino)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    # the first slice, and the last (ragged) slice of the batch
    for b in (0, B - 1):
        ref = obst.backproject(sino[b].double().cpu().numpy(), geom, obst.Params())
        err, worst = assert_parity(img[b].cpu().numpy(), ref)
        _say(f"[spb {spb}] slice {b}: rel-L2 {err:.2e}, max {worst:.2e}")
    # and bitwise the same as the default chunking, on every slice
    ref_plan = P.Plan(N, V, max_batch=B)
    assert torch.equal(img, ref_plan.backproject(sino))
    small = P.Plan(256, 301, max_batch=5, gather_slices=spb, filter="none")
    s2 = _sinos(5, 301, 256, 77)
    got = small.backproject(s2)
    g2 = Geometry(256, 301, 256)
    for b in range(5):
        assert_parity(got[b].cpu().numpy(), obst.backproject(s2[b].double().cpu().numpy(), g2,
                                                              obst.Params(filter="none")))


def test_largest_transform_4096(P):
    N, V = 4096, 48  # M = G = 8192: the row kernel's two-pairs-per-block path
    _say("[4096]")
    plan = P.Plan(N, V, max_batch=1)
    sino = _sinos(1, V, N, 4096, kind="plain")
    img = plan.backproject(sino)
    torch.cuda.synchronize()
    ref = obst.backproject(sino[0].double().cpu().numpy(), Geometry(N, V, N), obst.Params())
    assert rel_l2(img[0].cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("N,V,angles", [(16, 12, None), (64, 45, None), (256, 256, None),
                                        (128, 90, "random"), (32, 17, "random")])
def test_bruteforce_matches_oracle(P, N, V, angles):
    _say(f"[bruteforce] N={N} V={V} {angles}")
    rng = np.random.default_rng(N + V)
    th = None if angles is None else np.sort(rng.uniform(0, np.pi, V))
    plan = P.Plan(N, V, angles=th, max_batch=2)
    sino = _sinos(2, V, N, 3000 + N + V)
    img = plan.bruteforce(sino)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N, angles=th)
    for b in range(2):
        ref = obf.backproject(sino[b].double().cpu().numpy(), geom)
        assert rel_l2(img[b].cpu().numpy(), ref) <= 1e-5


def test_rotation_covariance_on_gpu(P):
    N, V = 256, 200
    plan = P.Plan(N, V, max_batch=2)
    y = _sinos(1, V, N, 77, kind="plain")[0].clone()
    y[:, 0] = 0.0
    h = V // 2
    yr = torch.zeros_like(y)
    yr[h:] = y[:h]
    yr[:h, 1:] = torch.flip(y[h:, 1:], dims=[1])
    out = plan.backproject(torch.stack([y, yr]))
    torch.cuda.synchronize()
    b, br = out[0].cpu().numpy(), out[1].cpu().numpy()
    expect = b[N - np.arange(1, N)].T
    assert rel_l2(br[:, 1:], expect) <= 1e-5


def test_deterministic_reruns(P):
    N, V, B = 512, 300, 4
    plan = P.Plan(N, V, max_batch=B)
    sino = _sinos(B, V, N, 99)
    ws = plan.workspace(B)
    a = plan.backproject(sino, workspace=ws).clone()
    b = plan.backproject(sino, workspace=ws).clone()
    c = plan.bruteforce(sino).clone()
    d = plan.bruteforce(sino).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(c, d)


def test_batch_slices_are_independent(P):
    """Slice b of a batch equals the same sinogram run alone (ragged last chunk of 16)."""
    N, V, B = 128, 100, 19
    plan = P.Plan(N, V, max_batch=B)
    sino = _sinos(B, V, N, 5)
    full = plan.backproject(sino)
    one = plan.backproject(sino[B - 1:B].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(full[B - 1], one[0])


@pytest.mark.parametrize("n,V", [(16, 5), (64, 33), (512, 64), (2048, 16)])
def test_ramp_filter_matches_oracle(P, n, V):
    # the brute-force FBP's ramp (Kak-Slaney kernel, linear convolution)
    plan = P.Plan(n, V, max_batch=2)
    sino = _sinos(2, V, n, 300 + n)
    q = plan.ramp_filter(sino)
    torch.cuda.synchronize()
    geom = Geometry(n, V, n)
    for b in range(2):
        y = sino[b].double().cpu().numpy()
        ref = oramp.filter_direct(y, geom.dt) if n <= 512 else oramp.filter_fft(y, geom.dt)
        assert_parity(q[b].cpu().numpy(), ref, tol=1e-6, elem=1e-6)


def test_gap_against_bruteforce_fbp(P):
    """Discretisation gap of the method (not a parity bar): BST FBP against
    brute-force FBP with the band-limited ramp, noiseless phantom, disk
    r <= (N/2 - 2) d."""
    N = 256
    sg = synth.Geometry(N, N, N)
    ell = synth.head_phantom(5, 10)
    y = synth.ellipse_sinogram(sg, ell).numpy()
    geom = Geometry(N, N, N)
    h = oramp.filter_fft(y, geom.dt)
    plan = P.Plan(N, N, max_batch=1)
    bst_img = plan.backproject(torch.tensor(y, dtype=torch.float32, device=DEV))
    bf_img = plan.bruteforce(torch.tensor(h, dtype=torch.float32, device=DEV))
    torch.cuda.synchronize()
    u = geom.u()
    disk = np.hypot(u[None, :], u[:, None]) <= (N / 2 - 2) * geom.d
    gap = rel_l2(bst_img.cpu().numpy()[disk], bf_img.cpu().numpy()[disk])
    _say(f"[gap] N={N}: {gap:.4f}")
    assert gap <= 3e-2


def test_gap_at_2048_meets_the_target(P):
    """The accuracy behind the benchmark's speed-ups: at the benchmark's size
    the default path (linear radial taps, P_c = 2) and the cubic-tap paths at
    P_c = 2 and 1 are within the 2e-2 target of brute-force FBP inside the
    disk, on a noiseless head phantom (the library's ramp filter, itself
    checked against the oracle, feeds the brute force)."""
    N = 2048
    sg = synth.Geometry(N, N, N)
    y = synth.ellipse_sinogram(sg, synth.head_phantom(5, 10), DEV).to(torch.float32).unsqueeze(0)
    lin = P.Plan(N, N)
    keys = P.Plan(N, N, taper="keys", interp="keys")
    keys1 = P.Plan(N, N, taper="keys", interp="keys", pad_cart=1)
    lin1 = P.Plan(N, N, pad_cart=1)
    bf = lin.bruteforce(lin.ramp_filter(y))
    imgs = {name: p.backproject(y) for name, p in (("linear", lin), ("keys", keys), ("keys_pc1", keys1),
                                                   ("linear_pc1", lin1))}
    torch.cuda.synchronize()
    u = (np.arange(N) - N // 2) * (2.0 / N)
    disk = np.hypot(u[None, :], u[:, None]) <= (N / 2 - 2) * (2.0 / N)
    ref = bf[0].cpu().numpy()[disk]
    gap = {name: rel_l2(img[0].cpu().numpy()[disk], ref) for name, img in imgs.items()}
    _say("[gap 2048] " + ", ".join(f"{k} {v:.4f}" for k, v in gap.items()))
    assert gap["linear"] <= 2e-2
    assert gap["keys"] <= 1e-2
    # cubic taps on the unoversampled grid (P_c = 1) still meet the target
    # (0.8 %); linear taps there do not (2.6 %)
    assert gap["keys_pc1"] <= 1e-2
    assert gap["linear_pc1"] > 2e-2


KEYS_CASES = [
    # N, V, filter, P_r, P_c: cubic radial interpolation with its de-apodiser
    (16, 10, "ramp", 2, 2),
    (16, 7, "none", 1, 1),
    (32, 24, "none", 2, 2),
    (64, 50, "ramp", 1, 2),
    (128, 96, "none", 4, 2),
    (256, 301, "ramp", 2, 2),
    (512, 400, "ramp", 2, 4),
    (2048, 2048, "ramp", 2, 2),
]


@pytest.mark.parametrize("N,V,filt,P_r,P_c", KEYS_CASES)
def test_keys_backproject_matches_oracle(P, N, V, filt, P_r, P_c):
    _say(f"[keys] N={N} V={V} {filt} Pr={P_r} Pc={P_c}")
    B = 2 if N < 2048 else 1
    plan = P.Plan(N, V, pad_radial=P_r, pad_cart=P_c, filter=filt, taper="keys", interp="keys", max_batch=B)
    sino = _sinos(B, V, N, 2500 + N + V)
    img = plan.backproject(sino)
    spec, dc = plan.debug_spectrum(sino)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(P_r, P_c, filt, "keys", interp="keys")
    M = P_r * N
    for b in range(B):
        y = sino[b].double().cpu().numpy()
        Yh, _ = obst.spectrum(y, geom, prm)
        assert rel_l2(spec[b].cpu().numpy(), Yh[:, :M // 2]) <= 1e-6
        ref = obst.backproject(y, geom, prm)
        err = rel_l2(img[b].cpu().numpy(), ref)
        _say(f"   slice {b}: rel-L2 {err:.2e}")
        assert err <= 1e-5


def _angle_set(kind, V, seed):
    rng = np.random.default_rng(seed)
    if kind == "jitter":
        th = (np.arange(V) + rng.uniform(-0.4, 0.4, V)) * np.pi / V
        th[0] = abs(th[0])
        return np.sort(th)
    if kind == "random":
        return np.sort(rng.uniform(0.0, np.pi, V))
    if kind == "clustered":   # two dense clusters and a wide gap, first angle above 0
        a = rng.uniform(0.2, 0.9, V // 2)
        b = rng.uniform(1.8, 2.9, V - V // 2)
        return np.sort(np.concatenate([a, b]))
    raise ValueError(kind)


NONUNIFORM_CASES = [
    # N, V, filter, P_r, P_c, angle set, interp
    (16, 11, "ramp", 2, 2, "random", "linear"),
    (64, 50, "none", 2, 2, "jitter", "linear"),
    (64, 40, "ramp", 1, 2, "clustered", "linear"),
    (128, 97, "ramp", 2, 2, "clustered", "keys"),
    (256, 256, "none", 2, 1, "random", "linear"),
    (512, 360, "ramp", 2, 2, "jitter", "keys"),
    (2048, 2048, "ramp", 2, 2, "jitter", "linear"),
]


@pytest.mark.parametrize("N,V,filt,P_r,P_c,kind,interp", NONUNIFORM_CASES)
def test_nonuniform_angles_match_oracle(P, N, V, filt, P_r, P_c, kind, interp):
    _say(f"[angles] N={N} V={V} {filt} Pr={P_r} Pc={P_c} {kind} {interp}")
    th = _angle_set(kind, V, 40 + N + V)
    assert np.all(np.diff(th) > 0) and th[0] >= 0 and th[-1] < np.pi
    B = 2 if N < 2048 else 1
    taper = "keys" if interp == "keys" else "deapod"
    plan = P.Plan(N, V, angles=th, pad_radial=P_r, pad_cart=P_c, filter=filt, taper=taper,
                  interp=interp, max_batch=B)
    sino = _sinos(B, V, N, 3000 + N + V)
    img = plan.backproject(sino)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N, angles=th)
    prm = obst.Params(P_r, P_c, filt, taper, interp=interp)
    for b in range(B):
        ref = obst.backproject(sino[b].double().cpu().numpy(), geom, prm)
        err = rel_l2(img[b].cpu().numpy(), ref)
        _say(f"   slice {b}: rel-L2 {err:.2e}")
        assert err <= 1e-5


def test_explicit_uniform_angles_match_the_uniform_plan(P):
    N, V = 256, 200
    sino = _sinos(2, V, N, 77)
    a = P.Plan(N, V, max_batch=2).backproject(sino)
    b = P.Plan(N, V, angles=np.arange(V) * np.pi / V, max_batch=2).backproject(sino)
    torch.cuda.synchronize()
    assert rel_l2(b.cpu().numpy(), a.cpu().numpy()) <= 2e-6


def test_keys_gap_against_bruteforce_fbp(P):
    """Cubic radial interpolation narrows the discretisation gap to brute-force
    FBP below 2 % at N = 256 (linear: ~2.3 %)."""
    N = 256
    sg = synth.Geometry(N, N, N)
    ell = synth.head_phantom(5, 10)
    y = synth.ellipse_sinogram(sg, ell).numpy()
    geom = Geometry(N, N, N)
    h = oramp.filter_fft(y, geom.dt)
    lin = P.Plan(N, N, max_batch=1)
    cub = P.Plan(N, N, max_batch=1, taper="keys", interp="keys")
    yt = torch.tensor(y, dtype=torch.float32, device=DEV)
    a = lin.backproject(yt)
    c = cub.backproject(yt)
    bf = lin.bruteforce(torch.tensor(h, dtype=torch.float32, device=DEV))
    torch.cuda.synchronize()
    u = geom.u()
    disk = np.hypot(u[None, :], u[:, None]) <= (N / 2 - 2) * geom.d
    bfn = bf.cpu().numpy()[disk]
    g_lin = rel_l2(a.cpu().numpy()[disk], bfn)
    g_cub = rel_l2(c.cpu().numpy()[disk], bfn)
    _say(f"[gap] N={N}: linear {g_lin:.4f}, keys {g_cub:.4f}")
    assert g_cub <= 2e-2
    assert g_cub < 0.8 * g_lin


def test_edge_cases(P):
    N, V = 64, 40
    plan = P.Plan(N, V, max_batch=4)
    sino = _sinos(4, V, N, 11)
    out = torch.full((4, N, N), 7.0, device=DEV)
    ws = plan.workspace(4)
    # batch 0: nothing enqueued, output untouched
    st = P.lib().bst_backproject(plan.handle, sino.data_ptr(), out.data_ptr(), 0, ws.data_ptr(),
                                 ws.numel(), None)
    assert st == 0
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    # workspace too small
    with pytest.raises(P.BstError) as e:
        plan.backproject(sino, out=out, workspace=ws[: ws.numel() // 2])
    assert e.value.status == 5
    assert torch.all(out == 7.0)
    # input/output overlap
    with pytest.raises(P.BstError) as e:
        flat = torch.empty(4 * V * N + 4 * N * N, device=DEV)
        st = P.lib().bst_backproject(plan.handle, flat.data_ptr(), flat.data_ptr() + 4 * 16,
                                     4, ws.data_ptr(), ws.numel(), None)
        P.binding._check(st, "bst_backproject")
    assert e.value.status == 10
    # batch above max
    big = _sinos(5, V, N, 12)
    with pytest.raises(P.BstError) as e:
        plan.backproject(big)
    assert e.value.status == 9
    # a plan built without adjoint tables has no projector: BST_E_UNSUPPORTED
    with pytest.raises(P.BstError) as e:
        plan.project(torch.zeros(1, N, N, device=DEV))
    assert e.value.status == 8
    # caller outputs must be exactly [B][N][N] (or [B][V][n]) float32: the library
    # takes no output size, so the binding refuses anything else before any call
    for bad in (torch.full((N, N), 7.0, device=DEV), torch.full((3, N, N), 7.0, device=DEV),
                torch.full((4, N, N), 7.0, device=DEV, dtype=torch.float64),
                torch.full((4, N, 2 * N), 7.0, device=DEV)[:, :, :N]):
        with pytest.raises((ValueError, TypeError)):
            plan.backproject(sino, out=bad, workspace=ws)
        with pytest.raises((ValueError, TypeError)):
            plan.bruteforce(sino, out=bad)
        assert torch.all(bad == 7.0)
    pa = P.Plan(N, V, max_batch=4, adjoint=True)
    for bad in (torch.zeros(V, N, device=DEV), torch.zeros(2, V, N, device=DEV)):
        with pytest.raises(ValueError):
            pa.project(torch.zeros(4, N, N, device=DEV), out=bad)
    # non-uniform angles: every path accepts them
    th = np.sort(np.random.default_rng(1).uniform(0, np.pi, V))
    p2 = P.Plan(N, V, angles=th, max_batch=1)
    out2 = p2.backproject(sino[0])
    p2.bruteforce(sino[0])
    torch.cuda.synchronize()
    assert math.isfinite(float(out.sum())) and math.isfinite(float(out2.sum()))
    assert P.Plan(N, V, angles=th, max_batch=1, adjoint=True).handle


# --- the adjoint projector and autograd ---------------------------------------

PROJ_CASES = [(16, 10, "ramp", 2, 2), (32, 21, "none", 1, 2), (64, 50, "ramp", 2, 1),
              (128, 96, "none", 2, 2), (256, 200, "ramp", 4, 2), (512, 300, "none", 2, 2)]


@pytest.mark.parametrize("N,V,filt,P_r,P_c", PROJ_CASES)
def test_project_matches_oracle(P, N, V, filt, P_r, P_c):
    _say(f"[project] N={N} V={V} {filt} Pr={P_r} Pc={P_c}")
    B = 3
    plan = P.Plan(N, V, pad_radial=P_r, pad_cart=P_c, filter=filt, max_batch=B, adjoint=True)
    g = torch.Generator(device="cpu")
    g.manual_seed(N + V)
    img = torch.randn(B, N, N, generator=g).to(DEV)
    out = plan.project(img)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(P_r, P_c, filt)
    for b in range(B):
        ref = obst.project(img[b].double().cpu().numpy(), geom, prm)
        err = rel_l2(out[b].cpu().numpy(), ref)
        _say(f"   slice {b}: rel-L2 {err:.2e}")
        assert err <= 1e-5


PROJ_OPTION_CASES = [
    # N, V, filter, P_r, P_c, interp, angle set (None = uniform)
    (32, 21, "ramp", 2, 2, "keys", None),
    (128, 96, "none", 2, 2, "keys", None),
    (64, 50, "ramp", 2, 2, "linear", "jitter"),
    (128, 97, "none", 1, 2, "linear", "clustered"),
    (256, 200, "ramp", 2, 2, "keys", "random"),
]


@pytest.mark.parametrize("N,V,filt,B,check", [
    (1024, 64, "none", 17, (0, 16)),   # G = 2048: 4 slices per round, two passes of paired rounds
    (2048, 32, "ramp", 1, (0,)),       # G = 4096: 2 slices per round, four passes
])
def test_project_large_grids_match_oracle(P, N, V, filt, B, check):
    """The column kernel's multi-pass path (grids of 2048 and 4096 points per
    side), with a ragged second slice group at 2048, against the oracle on
    sampled slices."""
    _say(f"[project-large] N={N} V={V} {filt} B={B}")
    plan = P.Plan(N, V, filter=filt, max_batch=B, adjoint=True)
    g = torch.Generator(device="cpu")
    g.manual_seed(N + V + B)
    img = torch.randn(B, N, N, generator=g).to(DEV)
    out = plan.project(img)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(2, 2, filt)
    for b in check:
        ref = obst.project(img[b].double().cpu().numpy(), geom, prm)
        err = rel_l2(out[b].cpu().numpy(), ref)
        _say(f"   slice {b}: rel-L2 {err:.2e}")
        assert err <= 1e-5


@pytest.mark.parametrize("N,V,filt,P_r,P_c,interp,kind", PROJ_OPTION_CASES)
def test_project_options_match_oracle(P, N, V, filt, P_r, P_c, interp, kind):
    """The projector for cubic radial interpolation and non-uniform angles
    (R = (d^2/dt) diag(1/w_j) B^T) against the oracle's transpose, and the
    weighted adjoint identity on the GPU."""
    _say(f"[project-opt] N={N} V={V} {filt} Pr={P_r} Pc={P_c} {interp} {kind}")
    th = None if kind is None else _angle_set(kind, V, 50 + N + V)
    B = 2
    taper = "keys" if interp == "keys" else "deapod"
    plan = P.Plan(N, V, angles=th, pad_radial=P_r, pad_cart=P_c, filter=filt, taper=taper,
                  interp=interp, max_batch=B, adjoint=True)
    g = torch.Generator(device="cpu")
    g.manual_seed(N + V + 5)
    img = torch.randn(B, N, N, generator=g).to(DEV)
    y = torch.randn(B, V, N, generator=g).to(DEV)
    out = plan.project(img)
    By = plan.backproject(y)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N, angles=th)
    prm = obst.Params(P_r, P_c, filt, taper, interp=interp)
    for b in range(B):
        ref = obst.project(img[b].double().cpu().numpy(), geom, prm)
        err = rel_l2(out[b].cpu().numpy(), ref)
        _say(f"   slice {b}: rel-L2 {err:.2e}")
        assert err <= 1e-5
        lhs = obf.inner_sino(out[b].double().cpu().numpy(), y[b].double().cpu().numpy(), geom)
        rhs = obf.inner_image(img[b].double().cpu().numpy(), By[b].double().cpu().numpy(), geom)
        assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


@pytest.mark.parametrize("filt", ["ramp", "none"])
def test_gpu_adjoint_identity(P, filt):
    N, V, B = 256, 180, 2
    plan = P.Plan(N, V, filter=filt, max_batch=B, adjoint=True)
    g = torch.Generator(device="cpu")
    g.manual_seed(3)
    f = torch.randn(B, N, N, generator=g).to(DEV)
    y = torch.randn(B, V, N, generator=g).to(DEV)
    Rf = plan.project(f).double().cpu().numpy()
    By = plan.backproject(y).double().cpu().numpy()
    torch.cuda.synchronize()
    d, dt, w = 2.0 / N, 2.0 / N, math.pi / V
    lhs = dt * w * float(np.sum(Rf * y.double().cpu().numpy()))
    rhs = d * d * float(np.sum(f.double().cpu().numpy() * By))
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


def test_project_deterministic_and_batch_independent(P):
    # 19 slices: one full group of interleaved slices and a ragged one
    N, V, B = 128, 100, 19
    plan = P.Plan(N, V, max_batch=B, adjoint=True)
    f = torch.randn(B, N, N, device=DEV)
    a = plan.project(f).clone()
    b = plan.project(f).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    for s in (0, 15, 16, B - 1):
        one = plan.project(f[s:s + 1].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(a[s], one[0])


def test_project_two_slice_groups_match_oracle(P):
    """A batch spanning two groups of interleaved slices, the second ragged,
    against the oracle slice by slice."""
    N, V, B = 64, 50, 19
    _say(f"[project-groups] N={N} V={V} B={B}")
    plan = P.Plan(N, V, max_batch=B, adjoint=True)
    g = torch.Generator(device="cpu")
    g.manual_seed(19)
    img = torch.randn(B, N, N, generator=g).to(DEV)
    out = plan.project(img).cpu().numpy()
    geom = Geometry(N, V, N)
    prm = obst.Params()
    for b in (0, 7, 15, 16, 18):
        ref = obst.project(img[b].double().cpu().numpy(), geom, prm)
        assert rel_l2(out[b], ref) <= 1e-5


@pytest.mark.parametrize("interp", ["linear", "keys"])
def test_autograd_gradients(P, interp):
    from paper_1704_08364_amd import autograd as AG
    N, V, B = 64, 48, 2
    plan = P.Plan(N, V, filter="none", max_batch=B, adjoint=True, interp=interp,
                  taper="keys" if interp == "keys" else "deapod")
    gen = torch.Generator(device="cpu")
    gen.manual_seed(5)
    f = torch.randn(B, N, N, generator=gen).to(DEV).requires_grad_(True)
    gs = torch.randn(B, V, N, generator=gen).to(DEV)
    v = torch.randn(B, N, N, generator=gen).to(DEV)

    def loss64(x):
        r = AG.project(x, plan).double() - gs.double()
        return float((r * r).sum())

    r = AG.project(f, plan) - gs
    loss = (r * r).sum()
    (grad,) = torch.autograd.grad(loss, f)
    # explicit form: 2 c B (R f - g)
    c = AG.adjoint_scale(plan)
    explicit = 2.0 * c * plan.backproject((plan.project(f.detach()) - gs).contiguous())
    assert rel_l2(grad.cpu().numpy(), explicit.cpu().numpy()) <= 1e-6
    # central finite difference along v (exact for a quadratic up to rounding)
    eps = 1e-2
    with torch.no_grad():
        fd = (loss64(f + eps * v) - loss64(f - eps * v)) / (2 * eps)
    dd = float((grad.double() * v.double()).sum())
    assert abs(fd - dd) <= 1e-3 * abs(dd)
    # backward of the backprojection: d/dsino <h, B sino> = B^T h = R h / c
    s = gs.clone().requires_grad_(True)
    h = torch.randn(B, N, N, generator=gen).to(DEV)
    (gsino,) = torch.autograd.grad((AG.backproject(s, plan) * h).sum(), s)
    expect = plan.project(h) / c
    assert rel_l2(gsino.cpu().numpy(), expect.cpu().numpy()) <= 1e-6


def _oracle_least_squares(sino, geom, prm, step, steps):
    """Gradient descent on ||R f - g||^2 from f = 0 in FP64 with the oracle's
    operators: the Euclidean gradient is 2 R^T (R f - g) = 2 c B (R f - g),
    c = d^2 / (dt pi / V), since R = c B^T (uniform angles)."""
    c = geom.d ** 2 / (geom.dt * math.pi / geom.V)
    f = np.zeros((geom.N, geom.N))
    losses = []
    for _ in range(steps):
        r = obst.project(f, geom, prm) - sino
        losses.append(float((r * r).sum()))
        f = f - step * 2.0 * c * obst.backproject(r, geom, prm)
    r = obst.project(f, geom, prm) - sino
    losses.append(float((r * r).sum()))
    return f, losses


def test_least_squares_matches_oracle(P):
    # 20 gradient steps through the autograd pair against the same iteration
    # in FP64 with the oracle's B and R (same step, same FP32 input bytes)
    from paper_1704_08364_amd import autograd as AG
    N, V, B, steps = 64, 64, 2, 20
    plan = P.Plan(N, V, filter="none", max_batch=B, adjoint=True)
    sino = synth.batch_sinograms(B, N, V, seed=21, device=DEV, noise=0.0)
    step = 1.0 / AG.lipschitz(plan, (B, N, N))
    f, losses = AG.least_squares(plan, sino, steps=steps, step=step)
    _say(f"[ls] losses {losses[0]:.3e} -> {losses[-1]:.3e}")
    # exact gradients and a step of 1/L: every step lowers the loss
    assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:]))
    geom = Geometry(N, V, N)
    prm = obst.Params(filter="none")
    tot = np.zeros(steps + 1)
    for b in range(B):
        ref, ref_losses = _oracle_least_squares(sino[b].double().cpu().numpy(), geom, prm, step, steps)
        err = rel_l2(f[b].double().cpu().numpy(), ref)
        _say(f"[ls] slice {b}: f_20 rel-L2 vs FP64 oracle iteration {err:.2e}")
        assert err <= 1e-4
        tot += np.array(ref_losses)
    # the loss trajectory is the sum over the batch
    assert np.max(np.abs(np.array(losses) - tot) / tot) <= 1e-4


# --- the FP64 gradient-check path ------------------------------------------------

F64_CASES = [
    # N, V, filter, P_r, P_c, taper, apodisation, centre shift
    (16, 10, "ramp", 2, 2, "deapod", "ramlak", 0.0),
    (32, 21, "none", 1, 2, "none", "ramlak", 0.0),
    (64, 48, "none", 2, 2, "deapod", "hann", 1.5),
    (128, 97, "ramp", 4, 2, "kaiser", "shepp", -2.25),
    (256, 256, "ramp", 2, 4, "deapod", "ramlak", 0.0),
    (512, 300, "none", 2, 2, "deapod", "cosine", 3.0),
]


@pytest.mark.parametrize("N,V,filt,P_r,P_c,taper,apod,shift", F64_CASES)
def test_fp64_backproject_and_project_match_oracle(P, N, V, filt, P_r, P_c, taper, apod, shift):
    _say(f"[f64] N={N} V={V} {filt} Pr={P_r} Pc={P_c} {taper} {apod} beta={shift}")
    B = 2
    plan = P.Plan(N, V, pad_radial=P_r, pad_cart=P_c, filter=filt, taper=taper, apodization=apod,
                  center_shift=shift, max_batch=B, dtype="f64")
    sino = _sinos(B, V, N, 5000 + N).double()
    img = torch.randn(B, N, N, generator=torch.Generator().manual_seed(N), dtype=torch.float64).to(DEV)
    got_b = plan.backproject(sino)
    got_r = plan.project(img)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(P_r, P_c, filt, taper if taper != "kaiser" else "kb", 8.0, apod=apod, center_shift=shift)
    for b in range(B):
        ref_b = obst.backproject(sino[b].cpu().numpy(), geom, prm)
        ref_r = obst.project(img[b].cpu().numpy(), geom, prm)
        eb, er = rel_l2(got_b[b].cpu().numpy(), ref_b), rel_l2(got_r[b].cpu().numpy(), ref_r)
        _say(f"   slice {b}: B {eb:.2e}, R {er:.2e}")
        assert eb <= 1e-12 and er <= 1e-12


def test_fp64_adjoint_identity(P):
    N, V, B = 128, 90, 2
    plan = P.Plan(N, V, filter="none", max_batch=B, dtype="f64")
    gen = torch.Generator().manual_seed(12)
    f = torch.randn(B, N, N, generator=gen, dtype=torch.float64).to(DEV)
    g = torch.randn(B, V, N, generator=gen, dtype=torch.float64).to(DEV)
    Rf, Bg = plan.project(f), plan.backproject(g)
    d, dt = 2.0 / N, 2.0 / N
    lhs = float((Rf * g).sum()) * dt * (math.pi / V)
    rhs = float((f * Bg).sum()) * d * d
    _say(f"[f64 adjoint] <Rf,g> {lhs:.15e} <f,Bg> {rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


@pytest.mark.parametrize("filt", ["none", "ramp"])
def test_fp64_gradient_central_differences(P, filt):
    # L(f) = ||R f - g||^2 is quadratic, so the central difference at eps =
    # 1e-3 equals the directional derivative up to FP64 rounding
    from paper_1704_08364_amd import autograd as AG
    N, V, B = 64, 48, 2
    plan = P.Plan(N, V, filter=filt, max_batch=B, dtype="f64")
    gen = torch.Generator().manual_seed(31)
    f = torch.randn(B, N, N, generator=gen, dtype=torch.float64).to(DEV).requires_grad_(True)
    g = torch.randn(B, V, N, generator=gen, dtype=torch.float64).to(DEV)
    r = AG.project(f, plan) - g
    loss = (r * r).sum()
    (grad,) = torch.autograd.grad(loss, f)

    def L(x):
        with torch.no_grad():
            rr = plan.project(x) - g
            return float((rr * rr).sum())

    eps = 1e-3
    for k in range(3):
        v = torch.randn(B, N, N, generator=gen, dtype=torch.float64).to(DEV)
        fd = (L(f.detach() + eps * v) - L(f.detach() - eps * v)) / (2 * eps)
        dd = float((grad * v).sum())
        _say(f"[f64 fd {filt}] direction {k}: fd {fd:.15e} autograd {dd:.15e} rel {abs(fd - dd) / abs(dd):.2e}")
        assert abs(fd - dd) <= 1e-8 * abs(dd)
    # the backprojection's backward pass too: d/dsino <h, B sino> = R h / c
    s = g.clone().requires_grad_(True)
    h = torch.randn(B, N, N, generator=gen, dtype=torch.float64).to(DEV)
    (gs,) = torch.autograd.grad((AG.backproject(s, plan) * h).sum(), s)
    c = AG.adjoint_scale(plan)
    assert rel_l2(gs.cpu().numpy(), (plan.project(h) / c).cpu().numpy()) <= 1e-13


def test_ls_gradient_against_bruteforce_tent(P):
    """The least-squares gradient through the BST pair, 2 c B (R f - g), against
    the brute-force one, 2 c B_d (R_d f - g) (pixel-driven projector and its
    transpose): with the tent angular rule the two objectives' gradients agree
    to the method's discretisation gap (bilinear transposed gridding is about
    10x off, see the oracle tests)."""
    N = V = 64
    sg = synth.Geometry(N, V, N)
    g = synth.ellipse_sinogram(sg, synth.head_phantom(5, 8))
    f = synth.ellipse_image(sg, synth.head_phantom(6, 8))
    plan = P.Plan(N, V, filter="none", adjoint=True, angular="tent")
    from paper_1704_08364_amd import autograd as AG
    fd = f.to(torch.float32).to(DEV).requires_grad_(True)
    gd = g.to(torch.float32).to(DEV)
    r = AG.project(fd, plan) - gd
    (grad,) = torch.autograd.grad((r * r).sum(), fd)
    geom = Geometry(N, V, N)
    c = AG.adjoint_scale(plan)
    f64, g64 = fd.detach().double().cpu().numpy(), gd.double().cpu().numpy()
    ref = 2 * c * obf.backproject(obf.project(f64, geom) - g64, geom)
    gap = rel_l2(grad.cpu().numpy(), ref)
    _say(f"[ls gradient vs brute force, tent] rel-L2 {gap:.4f}")
    assert gap <= 0.15


# --- apodised ramp, known centre shift, flat/dark normalisation ----------------

@pytest.mark.parametrize("N,V,filt,apod,shift", [(128, 100, "ramp", "hann", 2.5),
                                                 (64, 48, "none", "shepp", -1.25),
                                                 (256, 256, "ramp", "cosine", 7.0)])
def test_backproject_and_project_with_apodisation_and_shift(P, N, V, filt, apod, shift):
    _say(f"[apod/shift] N={N} V={V} {filt} {apod} {shift}")
    B = 2
    plan = P.Plan(N, V, filter=filt, apodization=apod, center_shift=shift, max_batch=B, adjoint=True)
    sino = _sinos(B, V, N, 500 + N)
    img = plan.backproject(sino)
    f = torch.randn(B, N, N, device=DEV)
    proj = plan.project(f)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(2, 2, filt, apod=apod, center_shift=shift)
    for b in range(B):
        assert rel_l2(img[b].cpu().numpy(), obst.backproject(sino[b].double().cpu().numpy(), geom, prm)) <= 1e-5
        assert rel_l2(proj[b].cpu().numpy(), obst.project(f[b].double().cpu().numpy(), geom, prm)) <= 1e-5


def test_backproject_counts(P):
    N, V, B = 256, 200, 3
    sino = _sinos(B, V, N, 900, kind="plain")
    gen = torch.Generator(device=DEV)
    gen.manual_seed(9)
    flat = 1000.0 + 100.0 * torch.rand(B, N, device=DEV, generator=gen)
    dark = 10.0 * torch.rand(B, N, device=DEV, generator=gen)
    ymax = float(sino.abs().max())
    counts = (dark[:, None, :] + (flat - dark)[:, None, :] * torch.exp(-sino / ymax)).contiguous()
    plan = P.Plan(N, V, max_batch=B)
    img = plan.backproject_counts(counts, flat, dark)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    for b in range(B):
        y = obst.normalize(counts[b].double().cpu().numpy(), flat[b].double().cpu().numpy(),
                           dark[b].double().cpu().numpy())
        assert rel_l2(img[b].cpu().numpy(), obst.backproject(y, geom, obst.Params())) <= 1e-5


# --- uneven-size batches (one graph launch) ------------------------------------

def _uneven(B_sizes, seed):
    from paper_1704_08364_amd import Batch
    batch = Batch(B_sizes)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    sinos = torch.empty(batch.sino_elems, dtype=torch.float32, device=DEV)
    for i, (n, v) in enumerate(B_sizes):
        batch.sino_view(sinos, i).copy_(synth.batch_sinograms(1, n, v, seed + i, device=DEV)[0])
    imgs = torch.zeros(batch.img_elems, dtype=torch.float32, device=DEV)
    return batch, sinos, imgs


def test_uneven_batch_matches_oracle_and_replays(P):
    sizes = [(64, 40), (128, 100), (64, 40), (256, 130), (128, 100), (64, 90), (256, 512), (128, 64)]
    batch, sinos, imgs = _uneven(sizes, 77)
    assert batch.classes() == 3                  # one class per detector size
    ws = batch.workspace()
    batch.backproject(sinos, imgs, ws)           # captures the graph
    torch.cuda.synchronize()
    first = imgs.clone()
    for i, (n, v) in enumerate(sizes):
        _say(f"[uneven] instance {i}: n={n} V={v}")
        ref = obst.backproject(batch.sino_view(sinos, i).double().cpu().numpy(), Geometry(n, v, n))
        assert rel_l2(batch.img_view(imgs, i).cpu().numpy(), ref) <= 1e-5
    # replays, with eager work and synchronisation in between, equal the first run
    for r in range(3):
        imgs.zero_()
        _ = (sinos * 2.0).sum()
        torch.cuda.synchronize()
        batch.backproject(sinos, imgs, ws)
        torch.cuda.synchronize()
        assert torch.equal(imgs, first), f"replay {r}"


def test_uneven_batch_of_64_distinct_angle_counts(P):
    """64 instances over three detector sizes, no two with the same angle
    count (odd and even, fewer and more angles than bins): each class's plan
    is built for its largest V and every slice runs with its own V. Every
    instance against the oracle, then a tuned run and replays against the
    first."""
    sizes = [((64, 128, 256)[i % 3], 24 + 7 * i) for i in range(64)]
    assert len({v for _, v in sizes}) == 64
    batch, sinos, imgs = _uneven(sizes, 1704)
    assert batch.classes() == 3
    ws = batch.workspace()
    batch.backproject(sinos, imgs, ws)
    torch.cuda.synchronize()
    first = imgs.clone()
    for i, (n, v) in enumerate(sizes):
        _say(f"[uneven 64] instance {i}: n={n} V={v}")
        ref = obst.backproject(batch.sino_view(sinos, i).double().cpu().numpy(), Geometry(n, v, n))
        assert_parity(batch.img_view(first, i).cpu().numpy(), ref)
    batch.tune(sinos, imgs, ws)
    for r in range(3):
        imgs.zero_()
        _ = (sinos * 2.0).sum()
        torch.cuda.synchronize()
        batch.backproject(sinos, imgs, ws)
        torch.cuda.synchronize()
        # the tuned grid sizes change which block takes an item, not its arithmetic
        assert torch.equal(imgs, first), f"tuned replay {r}"


def test_uneven_batch_with_the_largest_transform(P):
    """4096-bin instances (G = 8192: the row kernel's two-pairs-per-block path,
    one row group per work item) beside a small one, tuned, against the
    oracle."""
    sizes = [(4096, 64), (64, 50), (4096, 33)]
    batch, sinos, imgs = _uneven(sizes, 4096)
    ws = batch.workspace()
    batch.tune(sinos, imgs, ws)
    imgs.zero_()
    batch.backproject(sinos, imgs, ws)
    torch.cuda.synchronize()
    for i, (n, v) in enumerate(sizes):
        _say(f"[uneven 4096] instance {i}: n={n} V={v}")
        ref = obst.backproject(batch.sino_view(sinos, i).double().cpu().numpy(), Geometry(n, v, n))
        assert_parity(batch.img_view(imgs, i).cpu().numpy(), ref)


def test_uneven_batch_tuned(P):
    sizes = [(128, 96), (256, 200), (128, 96), (512, 300)]
    batch, sinos, imgs = _uneven(sizes, 91)
    ws = batch.workspace()
    batch.tune(sinos, imgs, ws)
    imgs.zero_()
    batch.backproject(sinos, imgs, ws)
    torch.cuda.synchronize()
    for i, (n, v) in enumerate(sizes):
        ref = obst.backproject(batch.sino_view(sinos, i).double().cpu().numpy(), Geometry(n, v, n))
        assert rel_l2(batch.img_view(imgs, i).cpu().numpy(), ref) <= 1e-5


# --- monopole subtraction (plain B) --------------------------------------------

MONO_CASES = [
    # N, V, P_r, P_c, width, centre shift, interp, angle set
    (16, 10, 2, 2, 0.5, 0.0, "linear", None),
    (64, 50, 2, 2, 0.4, 0.0, "linear", None),
    (64, 33, 1, 2, 0.3, 1.5, "linear", None),
    (128, 97, 2, 4, 0.4, -2.25, "keys", None),
    (256, 200, 4, 2, 0.6, 0.0, "linear", "jitter"),
    (512, 300, 2, 2, 0.4, 3.0, "keys", "random"),
]


@pytest.mark.parametrize("N,V,P_r,P_c,width,shift,interp,angles", MONO_CASES)
def test_monopole_matches_oracle(P, N, V, P_r, P_c, width, shift, interp, angles):
    _say(f"[monopole] N={N} V={V} Pr={P_r} Pc={P_c} s={width} beta={shift} {interp} {angles}")
    th = None if angles is None else _angle_set(angles, V, 60 + N)
    B = 2
    taper = "keys" if interp == "keys" else "deapod"
    plan = P.Plan(N, V, angles=th, pad_radial=P_r, pad_cart=P_c, filter="none", taper=taper, interp=interp,
                  center_shift=shift, monopole_width=width, max_batch=B)
    sino = _sinos(B, V, N, 5000 + N + V)
    img = plan.backproject(sino)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N, angles=th)
    prm = obst.Params(P_r, P_c, "none", taper, interp=interp, center_shift=shift, monopole=width)
    for b in range(B):
        ref = obst.backproject(sino[b].double().cpu().numpy(), geom, prm)
        err = rel_l2(img[b].cpu().numpy(), ref)
        _say(f"   slice {b}: rel-L2 {err:.2e}")
        assert err <= 1e-5


@pytest.mark.parametrize("P_r", [1, 2])
def test_monopole_with_counts_matches_oracle(P, P_r):
    # raw counts: the mass kernel and the spectrum kernel both normalise as they load
    N, V, B = 128, 90, 2
    sino = _sinos(B, V, N, 910, kind="plain")
    gen = torch.Generator(device=DEV)
    gen.manual_seed(11)
    flat = 1000.0 + 100.0 * torch.rand(B, N, device=DEV, generator=gen)
    dark = 10.0 * torch.rand(B, N, device=DEV, generator=gen)
    ymax = float(sino.abs().max())
    counts = (dark[:, None, :] + (flat - dark)[:, None, :] * torch.exp(-sino / ymax)).contiguous()
    plan = P.Plan(N, V, pad_radial=P_r, filter="none", monopole_width=0.4, max_batch=B)
    img = plan.backproject_counts(counts, flat, dark)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(P_r, 2, "none", "deapod", monopole=0.4)
    for b in range(B):
        y = obst.normalize(counts[b].double().cpu().numpy(), flat[b].double().cpu().numpy(),
                           dark[b].double().cpu().numpy())
        assert rel_l2(img[b].cpu().numpy(), obst.backproject(y, geom, prm)) <= 1e-5


def test_monopole_narrows_the_gap_to_bruteforce(P):
    # plain B of a phantom: the BST result with the monopole removed is within
    # 1% of the brute-force sum of Eq. 2 inside the disk; without it, ~3%
    N = V = 256
    geom = synth.Geometry(N, V, N)
    y = synth.ellipse_sinogram(geom, synth.head_phantom(3, 10)).float().to(DEV)[None]
    bf_plan = P.Plan(N, V, filter="none", max_batch=1)
    ref = bf_plan.bruteforce(y)[0].double().cpu().numpy()
    u = (np.arange(N) - N // 2) * (2.0 / N)
    disk = np.sqrt(u[None, :] ** 2 + u[:, None] ** 2) <= (N / 2 - 2) * (2.0 / N)

    def gap(img):
        return np.linalg.norm((img - ref)[disk]) / np.linalg.norm(ref[disk])

    plain = gap(bf_plan.backproject(y)[0].double().cpu().numpy())
    mono = gap(P.Plan(N, V, filter="none", monopole_width=0.4).backproject(y)[0].double().cpu().numpy())
    _say(f"[monopole gap] plain {plain:.4f} monopole {mono:.4f}")
    assert plain > 0.02 and mono < 0.01


def test_monopole_in_an_uneven_batch(P):
    from paper_1704_08364_amd import Batch
    sizes = [(64, 40), (128, 100), (64, 57)]
    batch = Batch(sizes, filter="none", monopole_width=0.4)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(5)
    sinos = torch.empty(batch.sino_elems, dtype=torch.float32, device=DEV)
    for i, (n, v) in enumerate(sizes):
        batch.sino_view(sinos, i).copy_(synth.batch_sinograms(1, n, v, 500 + i, device=DEV)[0])
    imgs = torch.zeros(batch.img_elems, dtype=torch.float32, device=DEV)
    ws = batch.workspace()
    for r in range(2):
        batch.backproject(sinos, imgs, ws)
        torch.cuda.synchronize()
        for i, (n, v) in enumerate(sizes):
            prm = obst.Params(filter="none", monopole=0.4)
            ref = obst.backproject(batch.sino_view(sinos, i).double().cpu().numpy(), Geometry(n, v, n), prm)
            assert rel_l2(batch.img_view(imgs, i).cpu().numpy(), ref) <= 1e-5, (r, i)


# --- tent angular rule ----------------------------------------------------------

TENT_CASES = [
    # N, V, filter, P_r, P_c
    (16, 12, "none", 2, 2),
    (32, 24, "none", 2, 2),
    (64, 50, "ramp", 2, 2),
    (128, 128, "none", 2, 4),
    (256, 300, "none", 1, 2),
    (512, 256, "ramp", 2, 2),
]


@pytest.mark.parametrize("N,V,filt,P_r,P_c", TENT_CASES)
def test_tent_backproject_and_project_match_oracle(P, N, V, filt, P_r, P_c):
    _say(f"[tent] N={N} V={V} {filt} Pr={P_r} Pc={P_c}")
    B = 2
    plan = P.Plan(N, V, pad_radial=P_r, pad_cart=P_c, filter=filt, angular="tent", max_batch=B, adjoint=True)
    sino = _sinos(B, V, N, 7000 + N + V)
    img = plan.backproject(sino)
    g = torch.Generator(device="cpu")
    g.manual_seed(N)
    f = torch.randn(B, N, N, generator=g).to(DEV)
    proj = plan.project(f)
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(P_r, P_c, filt, angular="tent")
    for b in range(B):
        eb = rel_l2(img[b].cpu().numpy(), obst.backproject(sino[b].double().cpu().numpy(), geom, prm))
        ep = rel_l2(proj[b].cpu().numpy(), obst.project(f[b].double().cpu().numpy(), geom, prm))
        _say(f"   slice {b}: backproject rel-L2 {eb:.2e}, project rel-L2 {ep:.2e}")
        assert eb <= 1e-5 and ep <= 1e-5


def test_tent_slice_groups_match_oracle(P):
    """The pre-gather's radius-major copy holds the slices in interleaved
    groups: a batch spanning several groups, the last ragged, against the
    oracle slice by slice, and each sampled slice equal to its own one-slice
    run."""
    N, V, B = 64, 64, 19
    _say(f"[tent-groups] N={N} V={V} B={B}")
    plan = P.Plan(N, V, angular="tent", max_batch=B)
    sino = _sinos(B, V, N, 7019)
    img = plan.backproject(sino).clone()
    torch.cuda.synchronize()
    geom = Geometry(N, V, N)
    prm = obst.Params(angular="tent")
    for b in (0, 9, 15, 16, 18):
        ref = obst.backproject(sino[b].double().cpu().numpy(), geom, prm)
        assert rel_l2(img[b].cpu().numpy(), ref) <= 1e-5
        one = plan.backproject(sino[b:b + 1].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(img[b], one[0])


def test_tent_projector_approximates_the_radon_transform(P):
    # the adjoint of the tent gather is a close Radon approximation, unlike the
    # adjoint of the bilinear gather (which over-weights lattice angles)
    N = V = 256
    geom = synth.Geometry(N, V, N)
    ell = synth.head_phantom(4, 8)
    f = synth.ellipse_image(geom, ell).float().to(DEV)[None]
    radon = synth.ellipse_sinogram(geom, ell).numpy()

    def err(**kw):
        plan = P.Plan(N, V, filter="none", adjoint=True, **kw)
        y = plan.project(f)[0].double().cpu().numpy()
        return np.linalg.norm(y - radon) / np.linalg.norm(radon)

    e_tent, e_lin = err(angular="tent"), err()
    _say(f"[tent radon] tent {e_tent:.4f} linear {e_lin:.3f}")
    assert e_tent < 0.1 and e_lin > 2.0


def test_tent_adjoint_identity_and_least_squares(P):
    from paper_1704_08364_amd import autograd as AG
    N, V, B = 128, 128, 2
    plan = P.Plan(N, V, filter="none", angular="tent", max_batch=B, adjoint=True)
    g = torch.Generator(device="cpu")
    g.manual_seed(17)
    f = torch.randn(B, N, N, generator=g).to(DEV)
    y = torch.randn(B, V, N, generator=g).to(DEV)
    geom = Geometry(N, V, N)
    Rf = plan.project(f).double().cpu().numpy()
    By = plan.backproject(y).double().cpu().numpy()
    for b in range(B):
        lhs = obf.inner_sino(Rf[b], y[b].double().cpu().numpy(), geom)
        rhs = obf.inner_image(f[b].double().cpu().numpy(), By[b], geom)
        # FP32 sums of random data cancel: the same 1e-5 as the bilinear identity test
        assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs))
    # least squares against analytic sinograms: with the tent the forward
    # model is the Radon transform, so the iterates approach the phantom
    sgeom = synth.Geometry(N, V, N)
    ells = [synth.head_phantom(30 + b, 8) for b in range(B)]
    truth = torch.stack([synth.ellipse_image(sgeom, e) for e in ells]).float().to(DEV)
    sino = torch.stack([synth.ellipse_sinogram(sgeom, e) for e in ells]).float().to(DEV)
    errs = {}
    for kind in ("tent", "linear"):
        pl = P.Plan(N, V, filter="none", angular=kind, max_batch=B, adjoint=True)
        rec, losses = AG.least_squares(pl, sino, steps=20)
        assert all(b <= a * (1 + 1e-6) for a, b in zip(losses, losses[1:]))
        errs[kind] = float((rec - truth).norm() / truth.norm())
    _say(f"[tent ls] image error after 20 steps: tent {errs['tent']:.3f} linear {errs['linear']:.3f}")
    assert errs["tent"] < 0.5 * errs["linear"]


def test_tent_in_an_uneven_batch(P):
    from paper_1704_08364_amd import Batch
    sizes = [(64, 40), (128, 100), (64, 40)]
    batch = Batch(sizes, angular="tent")
    sinos = torch.empty(batch.sino_elems, dtype=torch.float32, device=DEV)
    for i, (n, v) in enumerate(sizes):
        batch.sino_view(sinos, i).copy_(synth.batch_sinograms(1, n, v, 800 + i, device=DEV)[0])
    imgs = torch.zeros(batch.img_elems, dtype=torch.float32, device=DEV)
    ws = batch.workspace()
    for r in range(2):
        batch.backproject(sinos, imgs, ws)
        torch.cuda.synchronize()
        for i, (n, v) in enumerate(sizes):
            ref = obst.backproject(batch.sino_view(sinos, i).double().cpu().numpy(), Geometry(n, v, n),
                                   obst.Params(angular="tent"))
            assert rel_l2(batch.img_view(imgs, i).cpu().numpy(), ref) <= 1e-5, (r, i)


# --- the options at the benchmark's size ---------------------------------------

@pytest.mark.parametrize("option", ["keys", "tent", "monopole"])
def test_options_at_2048(P, option):
    # one 2048 x 2048-angle slice per option against the oracle, in a plan
    # sized for the 64-slice batch the benchmark times
    N = V = 2048
    kw, okw = {}, {}
    if option == "keys":
        kw, okw = dict(interp="keys", taper="keys"), dict(interp="keys", taper="keys")
    elif option == "tent":
        kw, okw = dict(angular="tent"), dict(angular="tent")
    else:
        kw, okw = dict(filter="none", monopole_width=0.4), dict(filter="none", monopole=0.4)
    _say(f"[2048] {option}")
    plan = P.Plan(N, V, max_batch=64, **kw)
    sino = _sinos(2, V, N, 9100)
    img = plan.backproject(sino)
    torch.cuda.synchronize()
    ref = obst.backproject(sino[1].double().cpu().numpy(), Geometry(N, V, N), obst.Params(**okw))
    err = rel_l2(img[1].cpu().numpy(), ref)
    _say(f"   rel-L2 {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("option", ["tent", "monopole", "keys"])
def test_options_are_deterministic_and_batch_independent(P, option):
    """Reruns are bitwise equal, and a slice's image does not depend on the
    batch around it (the tent pre-gather works in groups of 8 slices, the
    monopole mass from per-slice partial sums)."""
    N, V, B = 128, 100, 11
    kw = {"tent": dict(angular="tent"), "monopole": dict(filter="none", monopole_width=0.4),
          "keys": dict(interp="keys", taper="keys")}[option]
    plan = P.Plan(N, V, max_batch=B, **kw)
    sino = _sinos(B, V, N, 33)
    a = plan.backproject(sino)
    b = plan.backproject(sino)
    alone = plan.backproject(sino[9:10].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a[9], alone[0])


def test_tent_with_monopole_shift_and_apodisation(P):
    # every pre- and post-pass of the plain-B path in one plan
    N, V, B = 256, 240, 3
    plan = P.Plan(N, V, filter="none", angular="tent", monopole_width=0.45, center_shift=1.75,
                  apodization="hann", max_batch=B)
    sino = _sinos(B, V, N, 4242)
    img = plan.backproject(sino)
    torch.cuda.synchronize()
    prm = obst.Params(filter="none", angular="tent", monopole=0.45, center_shift=1.75, apod="hann")
    for b in range(B):
        ref = obst.backproject(sino[b].double().cpu().numpy(), Geometry(N, V, N), prm)
        assert rel_l2(img[b].cpu().numpy(), ref) <= 1e-5
