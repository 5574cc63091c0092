#!/usr/bin/env python3
"""Benchmark: BST filtered backprojection of 64 slices x 2048 angles x 2048 bins
-> 64 x 2048 x 2048 on one MI355X.

A step is one bst_backproject call over the whole batch (spectrum kernel,
gather + column inverse FFT kernel, row C2R kernel), with the sinograms already
resident in HBM. Prints one JSON line with slices/s, the roofline of the
dominant kernel measured with HIP events on the launch stream, the GPU
brute-force backprojection on the same sinograms, and the FP64 CPU oracle
timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "BST slices/s at N=2048, 2048 angles vs GPU brute-force BP at rel-L2 ≤ 1e-5"
HBM_PEAK_GBS = 8000.0
KERNELS = ("k_spectrum", "k_gather_colifft", "k_row_c2r")
_KERNEL_HEADERS = ["fft_lds.h", "bst_internal.h", "bst_check.h", "monopole.h"]
KERNEL_SOURCES = {
    "k_spectrum": ["k_spectrum.hip"] + _KERNEL_HEADERS,
    "k_gather_colifft": ["k_gather_colifft.hip"] + _KERNEL_HEADERS,
    "k_row_c2r": ["k_row_c2r.hip"] + _KERNEL_HEADERS,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """Source text without comments and blank space: edits to comments do
    not change the kernel a counter run measured."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_sha(name: str) -> str:
    """Hash of the code (comments left out) of a kernel's source and headers."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[name]:
        with open(os.path.join(ROOT, "paper_1704_08364_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def algorithmic_bytes(B: int, n: int, V: int, N: int, M: int, G: int) -> dict:
    """Minimum HBM bytes each kernel must move per launch (each input read once,
    each output written once)."""
    sino = B * V * n * 4
    polar = B * V * (M // 2) * 8 + B * V * 4          # spectrum + DC terms
    grid = B * N * (G // 2) * 8
    img = B * N * N * 4
    return {
        "k_spectrum": sino + polar,
        "k_gather_colifft": polar + grid,
        "k_row_c2r": grid + img,
    }


def copy_bandwidth(dev, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + written per second) of a plain
    torch copy of nbytes, median of reps: the practical ceiling of a streaming
    kernel, reported beside the 8 TB/s peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 2 * nbytes / sorted(ts)[len(ts) // 2]


def measured_traffic(kernel: str, config_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            data = json.load(fh)
        ent = data.get(kernel, {}).get(config_key)
        if not ent or ent.get("source_sha") != kernel_source_sha(kernel):
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_slice(args):
    """One FP64 oracle backprojection (a process-pool task)."""
    from oracle import bst as obst
    from oracle.geometry import Geometry
    y, n, V, N, kw = args
    return obst.backproject(y, Geometry(n, V, N), obst.Params(**kw))


def cpu_baseline(sino_cpu, out_gpu_cpu, n, V, N, slices, interp="linear", filter="ramp", monopole=0.0,
                 angular="linear", pad_radial=2, pad_cart=2, workers=None):
    """The FP64 oracle, unchanged, on `slices` slices of the same batch, the
    slices spread over a pool of host processes (one oracle call each)."""
    import multiprocessing
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor

    # the host's share of cores (16 per GPU on the benchmark machines); fresh
    # interpreters ("spawn"), since this process holds the GPU
    workers = workers or min(16, len(os.sched_getaffinity(0)))
    kw = dict(filter=filter, monopole=monopole, angular=angular, pad_radial=pad_radial, pad_cart=pad_cart)
    if interp == "keys":
        kw.update(taper="keys", interp="keys")
    tasks = [(sino_cpu[i], n, V, N, kw) for i in range(slices)]
    with ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        list(ex.map(_oracle_slice, tasks[:workers], timeout=600))  # start-up and imports, not timed
        t0 = time.perf_counter()
        refs = list(ex.map(_oracle_slice, tasks, timeout=600))
        dt = time.perf_counter() - t0
    errs = [float(np.linalg.norm(out_gpu_cpu[i] - refs[i]) / np.linalg.norm(refs[i])) for i in range(slices)]
    return slices / dt, dt, errs, workers


def cpu_bruteforce_2048(sino_slice):
    """s/slice of the FP64 oracle's brute-force backprojection (B_d of Eq. 2)
    at 2048^2 from 2048 angles, one process, estimated from a band of 32 image
    rows (1/64 of the slice; the cost is the same for every pixel)."""
    import numpy as np

    from oracle import bruteforce as obf
    from oracle.geometry import Geometry

    n = sino_slice.shape[1]
    V = sino_slice.shape[0]
    rows = np.repeat(np.arange(n // 2 - 16, n // 2 + 16), n)
    cols = np.tile(np.arange(n), 32)
    t0 = time.perf_counter()
    obf.backproject_pixels(sino_slice, Geometry(n, V, n), rows, cols)
    return round((time.perf_counter() - t0) * (n * n) / rows.size, 2)


def cpu_small_case():
    """s/slice of the FP64 oracle's BST and brute-force backprojection (B_d of
    Eq. 2) at N = 256 (256 angles, one process): the single-slice case the
    oracle finishes in seconds."""
    import numpy as np

    import synth
    from oracle import bruteforce as obf
    from oracle import bst as obst
    from oracle.geometry import Geometry

    y, _, _ = synth.config1_sinogram()
    y = y.double().numpy()
    geom = Geometry(256, 256, 256)
    t0 = time.perf_counter()
    obst.backproject(y, geom, obst.Params())
    t1 = time.perf_counter()
    obf.backproject(y, geom)
    t2 = time.perf_counter()
    return {"n": 256, "bst_fp64_s_per_slice": round(t1 - t0, 4), "bruteforce_fp64_s_per_slice": round(t2 - t1, 4),
            "cores": 1}


GAP_TARGET = 2e-2


def disk_mask(N: int):
    """Pixels with r <= (N/2 - 2) d, the disk the method's gap is measured in."""
    import numpy as np
    u = (np.arange(N) - N // 2) * (2.0 / N)
    return np.hypot(u[None, :], u[:, None]) <= (N / 2 - 2) * (2.0 / N)


def gap_to_bruteforce(n: int, V: int, plans: dict) -> dict:
    """Discretisation gap of each plan: relative L2 inside the disk between its
    BST FBP and the brute-force FBP (the library's ramp filter, then the
    slant-stack sum of Eq. 2) of one noiseless 10-ellipse head phantom
    (analytic sinogram, FP64 then rounded to FP32)."""
    import numpy as np
    import torch

    import synth

    geom = synth.Geometry(n, V, n)
    y = synth.ellipse_sinogram(geom, synth.head_phantom(5, 10), "cuda:0").to(torch.float32).unsqueeze(0)
    ref_plan = next(iter(plans.values()))
    bf = ref_plan.bruteforce(ref_plan.ramp_filter(y))
    torch.cuda.synchronize()
    disk = disk_mask(n)
    b = bf[0].double().cpu().numpy()[disk]
    out = {}
    for name, plan in plans.items():
        img = plan.backproject(y)
        torch.cuda.synchronize()
        a = img[0].double().cpu().numpy()[disk]
        out[name] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return out


def volume_workload(args):
    """Full volume: 2048 slices x 2048 angles x 2048 bins (32 GiB in, 32 GiB out),
    sinograms of a seeded 30-ellipsoid phantom with Poisson-like noise at 1e5
    photons, all resident in HBM; BST FBP in batches of 64 with one plan."""
    import numpy as np
    import torch

    import paper_1704_08364_amd as P
    import synth

    S, n, V, Bt = args.slices, args.n, args.angles, args.batch
    N = n
    dev = "cuda:0"
    geom = synth.Geometry(n, V, N)
    params = synth.ellipsoid_volume_params(170408367, 30)
    log(f"generating the {S}-slice volume on the GPU ...")
    t0 = time.perf_counter()
    sino = torch.empty(S, V, n, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(170408367)
    for k in range(S):
        s_k = -1.0 + (k + 0.5) * 2.0 / S
        y = synth.ellipse_sinogram(geom, synth.ellipsoid_slice_ellipses(params, s_k), dev)
        sino[k] = synth.poisson_like_noise(y, 1e5, gen).to(torch.float32) if float(y.max()) > 0 else 0.0
        if k % 256 == 255:
            log(f"  {k + 1} slices")
    torch.cuda.synchronize()
    log(f"  {time.perf_counter() - t0:.1f} s")
    img = torch.empty(S, N, N, dtype=torch.float32, device=dev)
    kw = dict(taper="keys", interp="keys") if args.interp == "keys" else {}
    plan = P.Plan(n, V, max_batch=Bt, pad_radial=args.pad_radial, pad_cart=args.pad_cart, **kw)
    ws = plan.workspace(Bt)
    for b0 in range(0, min(S, Bt * args.warmup), Bt):
        plan.backproject(sino[b0:b0 + Bt], out=img[b0:b0 + Bt], workspace=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for b0 in range(0, S, Bt):
        plan.backproject(sino[b0:b0 + Bt], out=img[b0:b0 + Bt], workspace=ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    out = {"metric": "BST FBP of a full volume", "value": round(S / el, 2), "unit": "slices/s",
           "seconds": round(el, 4), "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{S} slices x {V} angles x {n} bins, 30-ellipsoid phantom, "
                                  f"Poisson-like noise 1e5 photons, batches of {Bt}", "slices": S,
                      "interp": args.interp, "pad_radial": args.pad_radial, "pad_cart": args.pad_cart}}
    if args.cpu_slices > 0:
        from oracle import bst as obst
        from oracle.geometry import Geometry
        errs = []
        for k in (S // 3, S // 2):
            prm = obst.Params(args.pad_radial, args.pad_cart, **kw)
            ref = obst.backproject(sino[k].double().cpu().numpy(), Geometry(n, V, N), prm)
            errs.append(float(np.linalg.norm(img[k].double().cpu().numpy() - ref) / np.linalg.norm(ref)))
        out["parity"] = {"slices_checked": 2, "max_rel_l2_vs_fp64_oracle": max(errs)}
    print(json.dumps(out), flush=True)


def ls_workload(args):
    """Least-squares reconstruction ||R f - g||^2 by 20 gradient steps from f = 0
    with the exact adjoint pair (autograd), 32 slices x 1024 angles x 1024 bins."""
    import torch

    import paper_1704_08364_amd as P
    from paper_1704_08364_amd import autograd as AG
    import synth

    B, n, V = args.batch, args.n, args.angles
    dev = "cuda:0"
    g = synth.batch_sinograms(B, n, V, seed=170408369, device=dev)
    plan = P.Plan(n, V, filter="none", max_batch=B, adjoint=True, angular=args.angular)
    step = 1.0 / AG.lipschitz(plan, (B, n, n))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f, losses = AG.least_squares(plan, g, steps=args.steps, step=step)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"metric": "least-squares gradient steps (forward R + backward B per step)",
           "value": round(args.steps / el, 3), "unit": "steps/s", "ms_per_step": round(el * 1e3 / args.steps, 3),
           "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "loss_first": losses[0], "loss_last": losses[-1],
           "config": {"workload": f"{B} slices x {V} angles x {n} bins, random ellipse phantoms",
                      "steps": args.steps, "angular": args.angular}}
    print(json.dumps(out), flush=True)


def uneven_workload(args):
    """Uneven-size batch: 512 sinograms, N drawn from {256, 512, 1024, 2048},
    n_angles uniform in [N/2, 2N], random 2D ellipse phantoms, one graph
    launch; the persistent grid sizes are tuned per size class and stage first."""
    import numpy as np
    import torch

    import paper_1704_08364_amd as P
    import synth

    rng = np.random.default_rng(170408368)
    count = args.count
    sizes = []
    for _ in range(count):
        n = int(rng.choice([256, 512, 1024, 2048]))
        sizes.append((n, int(rng.integers(n // 2, 2 * n + 1))))
    batch = P.Batch(sizes)
    dev = "cuda:0"
    sinos = torch.empty(batch.sino_elems, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(170408368)
    log(f"generating {count} uneven sinograms ...")
    for i, (n, v) in enumerate(sizes):
        batch.sino_view(sinos, i).copy_(torch.randn(v, n, device=dev, generator=gen)
                                        if args.input == "random" else
                                        synth.batch_sinograms(1, n, v, 170408368 + i, device=dev)[0])
    imgs = torch.empty(batch.img_elems, dtype=torch.float32, device=dev)
    ws = batch.workspace()
    t0 = time.perf_counter()
    batch.tune(sinos, imgs, ws)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    for _ in range(max(args.warmup, 1)):
        batch.backproject(sinos, imgs, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        batch.backproject(sinos, imgs, ws)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t1) / args.steps
    pix = sum(n * n for n, _ in sizes)
    out = {"metric": "uneven-size BST batch in one graph launch", "value": round(count / el, 2),
           "unit": "sinograms/s", "ms_per_step": round(el * 1e3, 3), "n_gpus": 1, "dtype": "f32",
           "data": "synthetic", "classes": batch.classes(), "tune_seconds": round(tune_s, 2),
           "equivalent_2048_slices_per_s": round(pix / (2048 * 2048) / el, 1),
           "config": {"workload": f"{count} sinograms, N in {{256,512,1024,2048}}, V uniform in [N/2, 2N]"}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--angles", type=int, default=2048)
    ap.add_argument("--cpu-slices", type=int, default=64,
                    help="slices the FP64 oracle times, spread over the host's cores")
    ap.add_argument("--bf-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bruteforce", action="store_true")
    ap.add_argument("--no-gap", action="store_true",
                    help="skip the gap to brute force and the cubic path's timing")
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--workload", choices=("batch", "volume", "ls", "uneven"), default="batch",
                    help="batch: 64 x 2048^2 FBP (default); volume: the full 2048^3 volume; "
                         "ls: 32 x 1024^2 least squares by gradient descent")
    ap.add_argument("--slices", type=int, default=2048)
    ap.add_argument("--interp", choices=("linear", "keys"), default="linear",
                    help="radial interpolation of the gather (keys: cubic, narrower gap to brute force)")
    ap.add_argument("--filter", choices=("ramp", "none"), default="ramp",
                    help="ramp: FBP (default); none: plain backprojection B y")
    ap.add_argument("--monopole", type=float, default=0.0,
                    help="with --filter none: subtract a Gaussian monopole of this width (units of t)")
    ap.add_argument("--angular", choices=("linear", "tent"), default="linear",
                    help="angular kernel of the gather (tent: widened at small radii; uniform angles, linear interp)")
    ap.add_argument("--input", choices=("phantom", "random"), default="phantom",
                    help="random: N(0,1) sinograms (for hardware-counter runs, where generating "
                         "phantoms with thousands of small kernels is slow)")
    ap.add_argument("--pad-radial", type=int, default=2, choices=(1, 2, 4),
                    help="radial zero padding P_r of step P2")
    ap.add_argument("--pad-cart", type=int, default=2, choices=(1, 2, 4),
                    help="Cartesian oversampling P_c of the gather grid")
    ap.add_argument("--gather-slices", type=int, default=0,
                    help="slices per block of the gather kernel (0: the library's default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy a 1 GiB buffer first, to scale FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: slices are independent, so a multi-GPU "
              "run is the single-GPU path on a slab of slices per GPU (no collectives); "
              "this benchmark measures one GPU (N=1).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "volume":
        return volume_workload(args)
    if args.workload == "ls":
        return ls_workload(args)
    if args.workload == "uneven":
        return uneven_workload(args)

    import numpy as np
    import torch

    import paper_1704_08364_amd as P
    import synth

    B, n, V = args.batch, args.n, args.angles
    N = n
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
    copy_gbs = copy_bandwidth(dev) / 1e9
    log(f"generating {B} sinograms {V}x{n} on the GPU ...")
    if args.input == "random":
        gen = torch.Generator(device=dev)
        gen.manual_seed(170408366)
        sino = torch.randn(B, V, n, device=dev, generator=gen)
    else:
        sino = synth.batch_sinograms(B, n, V, seed=170408366, device=dev)
    interp_kw = dict(taper="keys", interp="keys") if args.interp == "keys" else {}
    plan = P.Plan(n, V, max_batch=B, filter=args.filter, monopole_width=args.monopole, angular=args.angular,
                  gather_slices=args.gather_slices, pad_radial=args.pad_radial, pad_cart=args.pad_cart, **interp_kw)
    M, G = plan.M, plan.G
    ws = plan.workspace(B)
    img = torch.empty(B, N, N, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.backproject(sino, out=img, workspace=ws, stream=stream)
    torch.cuda.synchronize()

    K = args.steps
    evs = [[P.Event() for _ in range(4)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        plan.backproject(sino, out=img, workspace=ws, stream=stream, events=evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / K
    value = B * K / elapsed
    per_kernel_ms = {}
    for i, name in enumerate(KERNELS):
        per_kernel_ms[name] = float(np.mean([evs[k][i].elapsed_ms(evs[k][i + 1]) for k in range(K)]))
    log(f"BST: {ms_per_step:.3f} ms/step ({B} slices) = {value:.1f} slices/s; per kernel ms: "
        + ", ".join(f"{k} {v:.3f}" for k, v in per_kernel_ms.items()))

    alg = algorithmic_bytes(B, n, V, N, M, G)
    dom = max(per_kernel_ms, key=per_kernel_ms.get)
    achieved = alg[dom] / (per_kernel_ms[dom] * 1e-3) / 1e9
    config_key = f"B{B}_n{n}_V{V}_N{N}_M{M}_G{G}"
    traffic = measured_traffic(dom, config_key)
    kernels = {}
    for name in KERNELS:
        gbs = alg[name] / (per_kernel_ms[name] * 1e-3) / 1e9
        kernels[name] = {"ms": round(per_kernel_ms[name], 4), "alg_bytes": alg[name],
                         "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}

    # GPU brute-force backprojection on the same sinograms
    bf = None
    if not args.no_bruteforce and args.bf_steps > 0:
        out_bf = torch.empty_like(img)
        plan.bruteforce(sino, out=out_bf, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.bf_steps):
            plan.bruteforce(sino, out=out_bf, stream=stream)
        torch.cuda.synchronize()
        bf_elapsed = time.perf_counter() - t1
        bf_rate = B * args.bf_steps / bf_elapsed
        bf = {"value": round(bf_rate, 2), "unit": "slices/s",
              "ms_per_step": round(bf_elapsed * 1e3 / args.bf_steps, 3),
              "speedup_bst_over_bruteforce": round(value / bf_rate, 2)}
        log(f"brute force: {bf_rate:.2f} slices/s; BST speedup {value / bf_rate:.1f}x")
        del out_bf

    # The accuracy behind the speed-up: the gap to brute force, on a noiseless
    # phantom, of both radial interpolations at the Cartesian oversampling of
    # the run and at P_c = 1; the speed-up is quoted for the fastest
    # configuration within the 2e-2 target.
    accuracy = None
    if not args.no_gap and args.filter == "ramp" and args.monopole == 0.0 and args.angular == "linear":
        cands = {}
        for pc in dict.fromkeys((args.pad_cart, 1)):
            for interp in ("linear", "keys"):
                name = interp + ("" if pc == args.pad_cart else f"_pc{pc}")
                cands[name] = dict(interp=interp, pad_cart=pc)
        main_name = args.interp
        gaps, rates = {}, {}
        for name, c in cands.items():
            kw = dict(taper="keys", interp="keys") if c["interp"] == "keys" else {}
            cplan = plan if name == main_name else P.Plan(n, V, max_batch=B, gather_slices=args.gather_slices,
                                                           pad_radial=args.pad_radial, pad_cart=c["pad_cart"], **kw)
            gaps[name] = gap_to_bruteforce(n, V, {name: cplan})[name]
            if name == main_name:
                rates[name] = value
            else:
                cws = cplan.workspace(B)
                for _ in range(2):
                    cplan.backproject(sino, out=img, workspace=cws, stream=stream)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                for _ in range(K):
                    cplan.backproject(sino, out=img, workspace=cws, stream=stream)
                torch.cuda.synchronize()
                rates[name] = B * K / (time.perf_counter() - t2)
                del cws, cplan
        ok = [m for m in cands if gaps[m] <= GAP_TARGET]
        best = max(ok, key=lambda m: rates[m]) if ok else min(gaps, key=gaps.get)
        accuracy = {"gap_rel_l2_in_disk": {m: round(g, 5) for m, g in gaps.items()}, "target": GAP_TARGET,
                    "phantom": f"noiseless 10-ellipse head phantom, analytic sinogram, {V}x{n} -> {n}^2, "
                               f"disk r <= (N/2-2) d; brute force = Kak-Slaney ramp + Eq. 2 sum",
                    "slices_per_s": {m: round(r, 1) for m, r in rates.items()},
                    "matched": {"path": best, "interp": cands[best]["interp"], "pad_cart": cands[best]["pad_cart"],
                                "meets_target": bool(ok), "slices_per_s": round(rates[best], 1),
                                "speedup_over_bruteforce": round(rates[best] / bf["value"], 2) if bf else None}}
        log("gap to brute force: " + ", ".join(f"{m} {g:.4f}" for m, g in gaps.items())
            + f" (target {GAP_TARGET}); matched path {best}: {rates[best]:.0f} slices/s")
        plan.backproject(sino, out=img, workspace=ws, stream=stream)  # the checked output is the main path's
        torch.cuda.synchronize()

    cpu = None
    parity = None
    if not args.no_cpu_baseline and args.cpu_slices > 0:
        s = min(args.cpu_slices, B)
        sino_cpu = sino[:s].double().cpu().numpy()
        img_cpu = img[:s].double().cpu().numpy()
        log(f"timing the FP64 oracle on {s} slices ...")
        try:
            rate, dt, errs, workers = cpu_baseline(sino_cpu, img_cpu, n, V, N, s, args.interp, args.filter,
                                                   args.monopole, args.angular, args.pad_radial, args.pad_cart)
            cpu = {"value": round(rate, 4), "unit": "slices/s", "cores": workers, "kind": "oracle",
                   "sample": f"{s} of the {B} slices ({V}x{n} -> {N}^2), FP64 NumPy BST (the oracle as it "
                             f"stands), one slice per task over {workers} host processes, {dt:.1f} s",
                   "cpu_model": _cpu_model(), "small_case": cpu_small_case(),
                   "bruteforce_fp64_s_per_slice": cpu_bruteforce_2048(sino_cpu[0])}
            parity = {"slices_checked": s, "max_rel_l2_vs_fp64_oracle": max(errs)}
            log(f"oracle: {rate:.4f} slices/s on {workers} processes; GPU vs oracle rel-L2 {max(errs):.2e}")
        except Exception as exc:  # a reported baseline, not the product: keep the benchmark line
            log(f"CPU baseline failed: {exc!r}")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("FBP" if args.filter == "ramp" else "plain backprojection")
                        + f" of {B} slices x {V} angles x {n} bins -> {B} x {N}x{N}, "
                        f"random 5-20 ellipse phantoms + 1% noise, P_r={args.pad_radial}, P_c={args.pad_cart}, "
                        + ("cubic (Keys) radial interpolation + its de-apodiser" if args.interp == "keys"
                           else "de-apodising taper")
                        + (f", monopole subtraction (s = {args.monopole})" if args.monopole else "")
                        + (", tent angular rule" if args.angular == "tent" else ""),
            "batch": B, "n_det": n, "n_angles": V, "n_out": N, "pad_radial": args.pad_radial,
            "pad_cart": args.pad_cart,
            "filter": args.filter, "input": args.input, "interp": args.interp, "monopole_width": args.monopole,
            "angular": args.angular,
            "seed": 170408366,
        },
        "env": {"device": torch.cuda.get_device_name(0), "torch": torch.__version__, "hip": torch.version.hip,
                "host_cpus": os.cpu_count()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "device_copy_GBps": round(copy_gbs, 1)},
        "kernels": kernels,
        "bruteforce": bf,
        "accuracy": accuracy,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
