"""Throughput of the DT back-propagation + gridding hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dt_ewald_128]
                    [--method realspace|fourier [--variant 11|12] [--nsr X]]

One step = one full reconstruction (all views: contrast, DFT, eq. 11 filter,
propagation to every depth plane, inverse FFTs, trilinear gridding) of the
workload, images already resident in HBM, enqueued with tomo_reconstruct_async
(tomo_fourier_reconstruct_async for --method fourier); the K timed steps end with
one tomo_sync (domain errors of any step are still reported).  The time per step
with a synchronisation after every call is reported as ms_per_step_sync_each.
Prints one JSON line.  With
--method fourier a step is one reconstruction by the Fourier-space form instead
(spectra, 3D gridding of the filtered spectra, normalisation, inverse 3D FFT);
its throughput is quoted in the same unit (voxel*angle updates of the volume).

The roofline object is computed for the kernel with the largest share of the
step, from library-side HIP event timing (two events around every launch, on
the launch's stream) over a second timed region of the same K steps: its
algorithmic HBM bytes per launch over its average launch duration, against the
8 TB/s HBM peak.  Beside it: the whole step's algorithmic bytes against the same
peak, and for the plane kernel its FFT arithmetic (5 n log2 n per complex 2D FFT of
n = M^2 points, i.e. 2.5 log2(M^2) per voxel-angle update) against the FP32 vector
peak.  The CPU baseline is the FP64 oracle on the host's cores (its views split over
threads, partial sums added in order), over every view of the workload when that
fits the CPU budget (else a view subset), in the same run (rank 0, N = 1 only); the
same views give the rel-L2 of the GPU result against the oracle over all N^3 voxels.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
BF16_MFMA_PEAK = 2500.0          # TFLOP/s, dense BF16 matrix cores
FP32_VECTOR_PEAK = 157.3         # TFLOP/s, FP32 vector with packed FMA (256 CUs x 256 FLOP/clk x 2.4 GHz)
FP32_UNPACKED_PEAK = 78.6        # TFLOP/s, FP32 vector without packed instructions (how this library is built)
CPU_BUDGET_UPDATES = 4.0e8       # oracle sample: at most this many voxel-angle updates (all views of 128^3 x 180)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="dt_ewald_128",
                    help="dt_ewald_128 | ct_pct_64 | xray_jitter_256 | batch64 (64 uneven jobs in one graph) | "
                         "unet128 (training step of the artefact-correction network at 128^3) | "
                         "unet_pairs (the network trained on 2000 seeded 128^3 pairs, 30 vs 720 views, and "
                         "evaluated on 200 held-out pairs)")
    ap.add_argument("--pairs", type=int, default=0, help="unet_pairs: training pairs (0: 2000)")
    ap.add_argument("--held-out", type=int, default=0, help="unet_pairs: held-out pairs (0: 200)")
    ap.add_argument("--epochs", type=int, default=10, help="unet_pairs: passes over the training pairs")
    ap.add_argument("--angle-batch", type=int, default=0)
    ap.add_argument("--tune", type=int, default=1, choices=[0, 1, 2, 3, 4, 5],
                    help="gridding variant: 0 fixed, 1 autotuned at plan time (default), 2 cubic tiles, "
                         "3 / 4 / 5 near-axis box with 4 / 8 / 2 rows (general frames; single-axis "
                         "frames keep 8 rows for 2 to 4 and take 2 rows for 5)")
    ap.add_argument("--plane-dtype", default="f32", choices=["f32", "bf16", "fp16"],
                    help="storage type of the plane stacks (interpolation and sums stay FP32)")
    ap.add_argument("--cpu-voxels", type=int, default=0,
                    help="evaluate the oracle sample at this many seeded voxels (0: all voxels)")
    ap.add_argument("--cpu-views", type=int, default=0,
                    help="views in the oracle sample (0: all views when N^3 n fits the CPU budget, else a subset)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="host threads of the oracle (0: all, at most 16)")
    ap.add_argument("--method", default="realspace", choices=["realspace", "fourier"])
    ap.add_argument("--variant", type=int, default=11, choices=[11, 12], help="Fourier-space form: eq. 11 or 12")
    ap.add_argument("--nsr", type=float, default=0.0, help="Fourier-space noise filter level (0: off)")
    ap.add_argument("--fourier-mode", type=int, default=1, choices=[1, 2],
                    help="Fourier-space gridding: 1 plan-time operator (gather), 2 per-call atomic splat")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def copy_probe(mib: int):
    """A plain copy of known size, run under the same profiler command as the bench so
    that its FETCH_SIZE / WRITE_SIZE readings calibrate the counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 5}), flush=True)


def kernel_source_hash(method: str = "realspace") -> str:
    """Hash of the code of the kernel sources a method runs (real-space: the FFT, spectra,
    plane and gridding kernels; fourier: the FFT header and the Fourier-space kernels): //
    comments, trailing blanks and empty lines are left out, so that editing a comment does not
    orphan the stored counter summaries."""
    csrc = os.path.join(ROOT, "paper_2206_09151_amd", "csrc")
    if method == "fourier":
        files = ["fft.hpp", "geom.hpp", "fourier_kernels.hip"]
    elif method == "unet":
        files = ["unet_internal.hpp", "unet_kernels.hip", "unet_host.hip"]
    else:
        files = ["fft.hpp", "fft_kernels.hpp", "geom.hpp", "tomo_kernels.hip"] + \
            sorted(f for f in os.listdir(csrc) if f.startswith("fft_sizes"))
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def algorithmic_bytes(kind: str, w, nb: int, first_batch: bool, sbytes: int = 4, fourier_mode: int = 1,
                      entries: int = 0) -> float:
    """Compulsory HBM bytes of the launches of one kind in one step over nb views;
    sbytes = bytes per stored plane value; entries = non-zeros of the Fourier-space
    gridding operator."""
    N, M, K = w.n_vox, w.M, w.K
    P = N + (1 - N % 2)
    fft3 = 2 * (8.0 + 8.0) * N ** 3 + (8.0 + 4.0) * N ** 3     # three passes, the last writes the real part
    if kind == "fgrid":
        if fourier_mode == 1:   # operator entries + row offsets + spectra + S read, complex grid written
            return 8.0 * entries + 4.0 * P ** 3 + nb * 16.0 * M * M + 8.0 * N ** 3 + 8.0 * N ** 3
        return nb * 16.0 * M * M + 2 * 16.0 * P ** 3           # spectra read, accumulator cleared and updated
    if kind == "finverse":
        if fourier_mode == 1:
            return fft3
        return 16.0 * P ** 3 + 8.0 * N ** 3 + 8.0 * N ** 3 + fft3   # + normalisation pass
    if kind == "spectra":   # image read + filter table read + Q write (16 B per coefficient each)
        return nb * (4.0 * M * M + 16.0 * M * M + 16.0 * M * M)
    if kind == "planes":    # Q read once per view + plane stack write
        return nb * (16.0 * M * M + sbytes * M * K * M)
    if kind == "grid":      # plane stack read + volume write (+ read when accumulating)
        return nb * sbytes * M * K * M + (4.0 if first_batch else 8.0) * N ** 3
    raise KeyError(kind)


def plane_flops(w, nb: int) -> float:
    """Algorithmic FFT operations of the plane kernel over nb views: one complex 2D FFT of
    n = M^2 points per plane pair, 5 n log2 n (the radix-2 count), i.e. 2.5 log2(M^2) per
    voxel-angle update when K = M = N."""
    M = w.M
    npairs = (w.K + 1) // 2 if w.ewald else 1
    n = float(M) * M
    return nb * npairs * 5.0 * n * np.log2(n)


def path_bytes_per_update(w, sbytes: int) -> float:
    """Algorithmic HBM bytes of a whole reconstruction per voxel-angle update: per view the
    image read and the plane stack written and read, plus the volume written once."""
    per_view = 4.0 * w.M * w.M + 2.0 * sbytes * w.M * w.K * w.M
    return (w.n_views * per_view + 4.0 * w.n_vox ** 3) / (float(w.n_vox) ** 3 * w.n_views)


def host_threads(requested: int = 0) -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    n = max(1, min(16, n))
    return min(requested, n) if requested > 0 else n


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threaded(images, dirs, dist, geo, views, threads: int, voxels=None):
    """The oracle's sum over `views`, the views cut into contiguous chunks run in host
    threads (numpy releases the interpreter lock in its array work; BLAS held to one
    thread each), partial sums added in chunk order.  The oracle itself is unchanged."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    chunks = [c for c in np.array_split(np.asarray(views), min(threads, len(views))) if len(c)]
    with threadpool_limits(1):
        with ThreadPoolExecutor(len(chunks)) as ex:
            parts = list(ex.map(lambda c: oracle.reconstruct_views(images, dirs, dist, geo, views=c,
                                                                   voxels=voxels), chunks))
    out = parts[0]
    for p in parts[1:]:
        out = out + p
    return out


def read_traffic(kind: str, src_hash: str, workload: str, storage: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source for this workload and plane storage."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kind}_{workload}_{storage}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != src_hash:
        return None
    return d.get("bytes_per_launch")


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (got --gpus {args.gpus}); "
              "there is no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch64":
        run_batch(args)
        return
    if args.workload == "unet128":
        run_unet(args)
        return
    if args.workload == "unet_pairs":
        run_unet_pairs(args)
        return
    import torch
    from synth import workloads
    from paper_2206_09151_amd import tomo

    w = workloads.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    t0 = time.time()
    ph, dirs, dist, imgs64 = workloads.make_workload(w, device="cuda")
    imgs = imgs64.astype(np.float32)
    gen_s = time.time() - t0
    print(f"[bench] inputs {w.name}: {imgs.shape} generated in {gen_s:.1f}s", file=sys.stderr, flush=True)
    d_img = torch.from_numpy(imgs).to(dev)
    vol = torch.empty((w.n_vox,) * 3, dtype=torch.float32, device=dev)
    params = tomo.Params(n_vox=w.n_vox, n_angles=w.n_views, voxel_size=w.voxel, wavelength=w.wavelength,
                         sigma=w.sigma, epsilon=w.epsilon, n_pix=w.M, n_planes=w.K, ewald=w.ewald,
                         weight_mode=w.weight_mode, eps_sampling=w.eps_sampling, i_in=w.i_in,
                         angle_batch=args.angle_batch, fourier=args.fourier_mode if args.method == "fourier" else 0,
                         tune=args.tune,
                         plane_dtype={"f32": tomo.F32, "bf16": tomo.BF16, "fp16": tomo.F16}[args.plane_dtype])
    stream = torch.cuda.current_stream()
    plan = tomo.Plan(params, dirs, dist, stream=stream)
    batch = plan.batch
    fourier = args.method == "fourier"

    # A step is enqueued without a host round trip (tomo_reconstruct_async or
    # tomo_fourier_reconstruct_async); the K steps end with one tomo_sync, which still reports
    # a domain error of any of them.  The rate with a synchronisation after every call is
    # reported beside.
    def step():
        if fourier:
            plan.fourier_reconstruct_async(d_img, vol, variant=args.variant, nsr=args.nsr, stream=stream)
        else:
            plan.reconstruct_async(d_img, vol, stream=stream)

    def finish():
        plan.sync(stream)

    for _ in range(args.warmup):
        step()
    finish()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        step()
    finish()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ms = elapsed * 1e3 / args.steps
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        if fourier:
            plan.fourier_reconstruct(d_img, vol, variant=args.variant, nsr=args.nsr, stream=stream)
        else:
            plan.reconstruct(d_img, vol, stream=stream)
    torch.cuda.synchronize()
    ms_sync_each = (time.perf_counter() - t) * 1e3 / args.steps
    updates = float(w.n_vox) ** 3 * w.n_views
    value = updates / (ms * 1e-3)
    print(f"[bench] {ms:.3f} ms/step, {value:.4g} updates/s (batch {batch})", file=sys.stderr, flush=True)

    roofline = None
    kernels = None
    if not args.no_kernel_timing:
        plan.timing(True)
        plan.timing_read(reset=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            step()
        finish()
        torch.cuda.synchronize()
        ms_timed = (time.perf_counter() - t) * 1e3 / args.steps
        plan.timing(False)
        k = plan.timing_read(reset=True)
        n_batches = -(-w.n_views // batch)
        kernels = {}
        for kind, (tot, cnt) in k.items():
            if cnt == 0:
                continue
            # bytes of all launches of one step (the first batch writes V without reading it)
            sb = 4 if args.plane_dtype == "f32" else 2
            if kind == "spectra" or fourier:   # launches over all views per step
                step_bytes = algorithmic_bytes(kind, w, w.n_views, True, sb, args.fourier_mode,
                                               plan.fourier_entries)
                per_launch = step_bytes / cnt * args.steps
            else:
                step_bytes = sum(algorithmic_bytes(kind, w, min(batch, w.n_views - b * batch), b == 0, sb)
                                 for b in range(n_batches))
                per_launch = step_bytes / n_batches
            avg_ms = tot / cnt
            kernels[kind] = {"avg_ms": avg_ms, "launches_per_step": cnt / args.steps,
                             "ms_per_step": tot / args.steps,
                             "algorithmic_bytes_per_launch": per_launch,
                             "GBps": per_launch / (avg_ms * 1e-3) / 1e9}
        dom = max(kernels, key=lambda kk: kernels[kk]["ms_per_step"])
        src_hash = kernel_source_hash("fourier" if fourier else "realspace")
        achieved = kernels[dom]["GBps"]
        sb = 4 if args.plane_dtype == "f32" else 2
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": read_traffic(dom, src_hash, w.name, args.plane_dtype),
                    "ms_per_step_with_events": round(ms_timed, 4), "kernel_source_hash": src_hash}
        if not fourier:
            pb = path_bytes_per_update(w, sb)
            roofline["path"] = {"bytes_per_update": round(pb, 3), "achieved": round(pb * value / 1e9, 1),
                                "frac": round(pb * value / 1e9 / HBM_PEAK_GBS, 4)}
        if "planes" in kernels:
            # the plane kernel's FFT arithmetic beside its bytes: it is bound by vector
            # arithmetic and LDS exchanges more than by its HBM writes
            fl = sum(plane_flops(w, min(batch, w.n_views - b * batch)) for b in range(n_batches)) / n_batches
            tflops = fl / (kernels["planes"]["avg_ms"] * 1e-3) / 1e12
            kernels["planes"]["algorithmic_flops_per_launch"] = fl
            kernels["planes"]["TFLOPs"] = tflops
            roofline["planes_fft"] = {"achieved": round(tflops, 2), "unit": "TFLOP/s", "peak": FP32_VECTOR_PEAK,
                                      "frac": round(tflops / FP32_VECTOR_PEAK, 4),
                                      "peak_without_packed_fp32": FP32_UNPACKED_PEAK,
                                      "frac_without_packed_fp32": round(tflops / FP32_UNPACKED_PEAK, 4),
                                      "flops_per_launch": fl}
        print(f"[bench] kernels: {json.dumps(kernels)}", file=sys.stderr, flush=True)

    cpu = None
    rel_l2 = max_rel = None
    if not args.no_cpu and fourier:
        import oracle
        from threadpoolctl import threadpool_limits
        geo = oracle.Geometry(w.n_vox, w.M, w.K if w.ewald else 1, w.voxel, w.wavelength, w.sigma, w.epsilon,
                              ewald=w.ewald, weight_mode=w.weight_mode, eps_sampling=w.eps_sampling,
                              i_in=w.i_in)
        with threadpool_limits(1):
            t = time.perf_counter()
            ref = oracle.fourier_reconstruct(imgs.astype(np.float64), dirs, dist, geo, nsr=args.nsr,
                                             variant=args.variant)
            cpu_s = time.perf_counter() - t
        cpu = {"value": updates / cpu_s, "unit": "voxel*angle updates/s", "cores": 1, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"whole workload ({w.n_views} views, {w.n_vox}^3), {cpu_s:.1f} s "
                         "(numpy FP64 Fourier-space form, one thread)"}
        plan.fourier_reconstruct(d_img, vol, variant=args.variant, nsr=args.nsr, stream=stream)
        torch.cuda.synchronize()
        got = vol.cpu().numpy().astype(np.float64)
        rel_l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"[bench] oracle {cpu_s:.1f}s; rel-L2 {rel_l2:.3g}", file=sys.stderr, flush=True)
    elif not args.no_cpu:
        import oracle
        threads = host_threads(args.cpu_threads)
        nv = args.cpu_views or max(min(threads, w.n_views), int(CPU_BUDGET_UPDATES // float(w.n_vox) ** 3))
        nv = min(nv, w.n_views)
        views = np.arange(nv)
        geo = oracle.Geometry(w.n_vox, w.M, w.K if w.ewald else 1, w.voxel, w.wavelength, w.sigma, w.epsilon,
                              ewald=w.ewald, weight_mode=w.weight_mode, eps_sampling=w.eps_sampling,
                              i_in=w.i_in)
        vox = None
        if args.cpu_voxels:
            vox = np.random.default_rng(7).integers(0, w.n_vox, size=(args.cpu_voxels, 3))
        imgs64f = imgs.astype(np.float64)
        t = time.perf_counter()
        ref = oracle_threaded(imgs64f, dirs, dist, geo, views, threads, voxels=vox)
        cpu_s = time.perf_counter() - t
        nvox = w.n_vox ** 3 if vox is None else len(vox)
        cpu = {"value": float(nvox) * nv / cpu_s, "unit": "voxel*angle updates/s", "cores": threads,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": (f"{nv} of {w.n_views} views, " +
                          (f"full {w.n_vox}^3 volume" if vox is None else f"{nvox} seeded voxels") +
                          f", {cpu_s:.1f} s wall on {threads} threads (numpy FP64; views split over threads, "
                          "partial sums added in order; includes the plan-stage weights)")}
        if nv == w.n_views:
            # the timed path's own output (the last timed step wrote vol)
            plan.reconstruct(d_img, vol, stream=stream)
            torch.cuda.synchronize()
            got = vol.cpu().numpy().astype(np.float64)
        else:
            # the same views through the stage entry points, compared over all voxels
            part = torch.zeros_like(vol)
            st = torch.empty(plan.stack_shape(min(batch, nv)), dtype=plan.stack_dtype, device=dev)
            for first in range(0, nv, batch):
                nb = min(batch, nv - first)
                plan.backpropagate(d_img[first:first + nb].contiguous(), first, nb, st, stream=stream)
                plan.grid(st, first, nb, part, stream=stream)
            torch.cuda.synchronize()
            got = part.cpu().numpy().astype(np.float64)
        if vox is not None:
            got = got[vox[:, 0], vox[:, 1], vox[:, 2]]
        rel_l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        max_rel = float(np.abs(got - ref).max() / np.abs(ref).max())
        print(f"[bench] oracle {cpu_s:.1f}s on {nv} views, {threads} threads; rel-L2 {rel_l2:.3g}, "
              f"max {max_rel:.3g}", file=sys.stderr, flush=True)

    out = {
        "metric": "voxel*angle updates/s (DT backprop+gridding)",
        "method": args.method if not fourier else
        f"fourier_eq{args.variant}_{'operator' if args.fourier_mode == 1 else 'splat'}",
        "value": value,
        "unit": "voxel*angle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "ms_per_step_sync_each": ms_sync_each,
        "config": {"workload": w.name, "n_vox": w.n_vox, "n_pix": w.M, "n_planes": w.K, "grid_variant": plan.grid_rows,
                   "plane_storage": args.plane_dtype,
                   "n_views": w.n_views, "ewald": w.ewald, "weight_mode": w.weight_mode,
                   "angle_batch": batch, "updates_per_step": updates,
                   **({"fourier_mode": args.fourier_mode, "operator_entries": plan.fourier_entries,
                       "variant": args.variant, "nsr": args.nsr} if fourier else {})},
        "rel_l2_vs_fp64": rel_l2,
        "max_abs_err_rel_to_max_vs_fp64": max_rel,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _make_job(w):
    from synth import workloads
    ph, dirs, dist, imgs = workloads.make_workload(w)
    return dirs, dist, imgs.astype(np.float32)


def run_batch(args):
    """64 uneven jobs (N in {64..192}, 60-240 views, single-axis and sphere scans) as one
    recorded graph: a step is one launch of all jobs; value = total N^3 n of the jobs
    per second.  Per-kernel figures come from one eager pass over the jobs with the
    library's event timing."""
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    from synth import workloads
    jobs = workloads.batch_jobs()
    t0 = time.time()
    # inputs are drawn on host threads (numpy releases the interpreter lock in its array work),
    # so that the bench stays one process, also under a profiler
    data = []
    with threadpool_limits(1), ThreadPoolExecutor(host_threads()) as pool:
        for i in range(0, len(jobs), 16):
            data += list(pool.map(_make_job, jobs[i:i + 16]))
            print(f"[bench] batch64: {len(data)}/{len(jobs)} jobs generated in {time.time() - t0:.0f}s",
                  file=sys.stderr, flush=True)
    print(f"[bench] batch64: {len(jobs)} jobs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    import torch
    from paper_2206_09151_amd import tomo
    dev = torch.device("cuda:0")
    plans, imgs, vols = [], [], []
    for w, (dirs, dist, im) in zip(jobs, data):
        params = tomo.Params(n_vox=w.n_vox, n_angles=w.n_views, voxel_size=w.voxel, wavelength=w.wavelength,
                             sigma=w.sigma, epsilon=w.epsilon, ewald=w.ewald, weight_mode=w.weight_mode,
                             eps_sampling=w.eps_sampling, i_in=w.i_in, tune=1)
        plans.append(tomo.Plan(params, dirs, dist))
        imgs.append(torch.from_numpy(im).to(dev))
        vols.append(torch.empty((w.n_vox,) * 3, dtype=torch.float32, device=dev))
    batch = tomo.Batch(plans, imgs, vols)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        batch.launch(stream)
    batch.sync(stream)
    t = time.perf_counter()
    for _ in range(args.steps):
        batch.launch(stream)
    batch.sync(stream)
    ms = (time.perf_counter() - t) * 1e3 / args.steps
    updates = float(sum(w.updates for w in jobs))
    value = updates / (ms * 1e-3)
    print(f"[bench] batch64: {ms:.3f} ms/step, {value:.4g} updates/s", file=sys.stderr, flush=True)

    kernels = roofline = None
    if not args.no_kernel_timing:
        tot = {}
        for pl, w, im, v in zip(plans, jobs, imgs, vols):
            pl.timing(True)
            pl.timing_read(reset=True)
            pl.reconstruct(im, v, stream=stream)
            pl.timing(False)
            nb_all = -(-w.n_views // pl.batch)
            for kind, (ms_k, cnt) in pl.timing_read(reset=True).items():
                if cnt == 0:
                    continue
                if kind == "spectra":
                    b = algorithmic_bytes(kind, w, w.n_views, True)
                else:
                    b = sum(algorithmic_bytes(kind, w, min(pl.batch, w.n_views - i * pl.batch), i == 0)
                            for i in range(nb_all))
                a = tot.setdefault(kind, [0.0, 0, 0.0])
                a[0] += ms_k
                a[1] += cnt
                a[2] += b
        kernels = {k: {"ms_total_eager": v[0], "launches": v[1], "algorithmic_bytes": v[2],
                       "GBps": v[2] / (v[0] * 1e-3) / 1e9} for k, v in tot.items()}
        dom = max(kernels, key=lambda kk: kernels[kk]["ms_total_eager"])
        achieved = kernels[dom]["GBps"]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "note": "eager pass over the 64 jobs with library event timing (the graph holds no events)",
                    "kernel_source_hash": kernel_source_hash("realspace")}
        print(f"[bench] kernels: {json.dumps(kernels)}", file=sys.stderr, flush=True)

    cpu = rel_l2 = None
    if not args.no_cpu:
        import oracle
        j = min(range(len(jobs)), key=lambda k: jobs[k].updates)
        w = jobs[j]
        dirs, dist, im = data[j]
        nv = min(args.cpu_views, w.n_views)
        geo = oracle.Geometry(w.n_vox, w.M, w.K, w.voxel, w.wavelength, w.sigma, w.epsilon, ewald=w.ewald,
                              weight_mode=w.weight_mode, eps_sampling=w.eps_sampling, i_in=w.i_in)
        t = time.perf_counter()
        ref = oracle.reconstruct_views(im.astype(np.float64), dirs, dist, geo, views=np.arange(nv))
        cpu_s = time.perf_counter() - t
        cpu = {"value": float(w.n_vox) ** 3 * nv / cpu_s, "unit": "voxel*angle updates/s", "cores": 1,
               "kind": "oracle",
               "sample": f"job {j} (N={w.n_vox}, {w.geometry}): {nv} of {w.n_views} views, full volume, "
                         f"{cpu_s:.1f} s (numpy FP64, single thread)"}
        pl = plans[j]
        part = torch.zeros_like(vols[j])
        st = torch.empty(pl.stack_shape(min(pl.batch, nv)), dtype=torch.float32, device=dev)
        for first in range(0, nv, pl.batch):
            nb = min(pl.batch, nv - first)
            pl.backpropagate(imgs[j][first:first + nb].contiguous(), first, nb, st, stream=stream)
            pl.grid(st, first, nb, part, stream=stream)
        torch.cuda.synchronize()
        got = part.cpu().numpy().astype(np.float64)
        rel_l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    out = {
        "metric": "voxel*angle updates/s (DT backprop+gridding)",
        "method": "realspace_batch_graph",
        "value": value,
        "unit": "voxel*angle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch64", "jobs": len(jobs), "n_vox": sorted({w.n_vox for w in jobs}),
                   "views_range": [min(w.n_views for w in jobs), max(w.n_views for w in jobs)],
                   "updates_per_step": updates},
        "rel_l2_vs_fp64": rel_l2,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    batch.destroy()


def unet_flops_per_voxel() -> float:
    """Multiply-adds x 2 of one training step (forward, input gradients except the
    first layer's, weight gradients) per voxel of the full-resolution volume."""
    from synth import netinit
    levels = [0, 0, 1, 1, 2, 2, 1, 1, 0, 0, 0]          # resolution level of each layer
    fwd = bwd = 0.0
    for i, ((ci, co, k), lv) in enumerate(zip(netinit.LAYERS, levels)):
        macs = ci * co * k ** 3 / 8.0 ** lv
        fwd += macs
        bwd += macs * (2 if i > 0 else 1)
    return 2.0 * (fwd + bwd)


def unet_mfma_flops_per_voxel() -> float:
    """Matrix-core flops the network kernels execute per training step and full-resolution
    voxel: the FP32 activations are split into BF16 hi + lo, so the forward and input-gradient
    products run twice (hi and lo packed into K) and the weight gradient three times (hi hi,
    hi lo, lo hi); the first layer's weight gradient pads its 27 taps to 32.  The 1x1 output
    layer and the first layer's forward run on the vector ALUs and are not counted."""
    from synth import netinit
    levels = [0, 0, 1, 1, 2, 2, 1, 1, 0, 0, 0]
    total = 0.0
    for i, ((ci, co, k), lv) in enumerate(zip(netinit.LAYERS, levels)):
        if k != 3:
            continue
        macs = ci * co * 27 / 8.0 ** lv
        if ci % 16 == 0:
            total += 2 * macs * 2          # forward
            total += 2 * macs * 2          # input gradient (every 16-channel layer has one)
            total += 2 * macs * 3          # weight gradient
        else:                              # single input channel: weight gradient only
            total += 2 * macs * (32 / 27) * 3
    return total


def run_unet(args):
    """Training step (forward, MSE, backward, Adam) of the artefact-correction network on
    128^3 diffraction-tomography volumes: sparse (30-view) reconstructions against dense
    (720-view) ones of the same phantoms, both made by this library.  Reports voxels per
    second of training, the matrix-core roofline, and the held-out error ratio after the run."""
    import torch
    from synth import netinit, workloads
    from paper_2206_09151_amd import tomo, unet
    base = workloads.WORKLOADS["dt_ewald_128"]
    n = base.n_vox
    dev = torch.device("cuda:0")
    t0 = time.time()
    pairs = []
    for k in range(3):
        vols = []
        for nv in (30, 720):
            w = base.scaled(name=f"unet_pair{k}_{nv}", index=200 + k, n_views=nv)
            ph, dirs, dist, im = workloads.make_workload(w, device="cuda")
            plan = tomo.Plan(tomo.Params(n_vox=n, n_angles=nv, voxel_size=w.voxel, wavelength=w.wavelength,
                                         sigma=w.sigma, epsilon=w.epsilon, n_pix=w.M, n_planes=w.K), dirs, dist)
            v = torch.empty((n, n, n), device=dev)
            plan.reconstruct(torch.from_numpy(im.astype(np.float32)).to(dev), v)
            plan.destroy()
            vols.append(v)
        pairs.append(tuple(vols))
    scale = float(torch.sqrt(torch.stack([(d * d).mean() for _, d in pairs]).mean()))
    pairs = [(a / scale, b / scale) for a, b in pairs]
    print(f"[bench] unet128: 3 pairs (30 vs 720 views) in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    train, held = pairs[:2], pairs[2]
    net = unet.Net(n)
    theta = torch.from_numpy(netinit.init_params(9)).to(dev)
    m, v, g = torch.zeros_like(theta), torch.zeros_like(theta), torch.empty_like(theta)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    step = 0

    def train_step():
        nonlocal step
        step += 1
        a, b = train[(step - 1) % len(train)]
        net.gradient(theta, a, b, g, loss)
        net.adam(theta, g, m, v, step, 1e-3)

    for _ in range(args.warmup):
        train_step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        train_step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / args.steps
    y = torch.empty((n, n, n), device=dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        net.forward(theta, held[0], y)
    torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t) * 1e3 / 5
    base_err = float(((held[0] - held[1]) ** 2).mean())
    corr_err = float(((y - held[1]) ** 2).mean())
    flops = unet_flops_per_voxel() * n ** 3
    useful = flops / (ms * 1e-3) / 1e12
    achieved = unet_mfma_flops_per_voxel() * n ** 3 / (ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu:
        import oracle.unet as ou
        crop = held[0][:32, :32, :32].cpu().numpy().astype(np.float64)
        tgt = held[1][:32, :32, :32].cpu().numpy().astype(np.float64)
        th = theta.cpu().numpy().astype(np.float64)
        tc = time.perf_counter()
        yo, cache = ou.forward(th, crop, bf16=True)
        _, gy = ou.mse(yo, tgt)
        ou.backward(th, cache, gy, bf16=True)
        cs = time.perf_counter() - tc
        cpu = {"value": 32.0 ** 3 / cs, "unit": "training voxels/s", "cores": 1, "kind": "oracle",
               "sample": f"one forward+backward of the FP64 oracle on a 32^3 crop, {cs:.1f} s (numpy)"}
    out = {
        "metric": "network training voxels/s (artefact correction, forward+backward+Adam)",
        "method": "unet_training",
        "value": n ** 3 / (ms * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 weights, f32 activations and sums", "data": "synthetic",
        "config": {"workload": "unet128", "n_vox": n, "params": unet.param_count(), "sparse_views": 30,
                   "dense_views": 720, "train_pairs": 2, "forward_ms": ms_fwd,
                   "heldout_mse_ratio_after_run": corr_err / base_err},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": BF16_MFMA_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / BF16_MFMA_PEAK, 4), "traffic": None,
                     "useful_fp32_equivalent_tflops": round(useful, 2),
                     "note": "BF16 matrix-core flops the convolutions execute per step (hi/lo split "
                             "included) / whole step time, against the dense BF16 peak",
                     "kernel_source_hash": kernel_source_hash("unet")},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    net.destroy()


def run_unet_pairs(args):
    """The artefact-correction network at its stated scale: 2000 training and 200 held-out
    seeded phantoms (ellipsoids, 128^3, the dt_ewald_128 physics), each reconstructed by this
    library from 30 views (input) and from 720 views (target; the 30 are every 24th of the
    720).  Trains for --epochs passes (one pair per Adam step, seeded shuffle, learning rate
    1e-3 then cosine-decayed to 1e-4 over the second half) and reports the held-out mean
    squared error against the dense reconstruction, of the network output and of the plain
    sparse reconstruction; the network is used only where it beats the plain reconstruction
    on the held-out set (else the plain reconstruction is the fallback)."""
    import torch
    from synth import learning, netinit, scan, workloads
    from paper_2206_09151_amd import tomo, unet
    base = workloads.WORKLOADS["dt_ewald_128"]
    n = base.n_vox
    n_train = args.pairs or learning.TRAIN
    n_held = args.held_out or learning.HELD_OUT
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    dirs = scan.single_axis(learning.DENSE_VIEWS, 180.0)
    dist = np.full(learning.DENSE_VIEWS, base.dist)
    step = learning.DENSE_VIEWS // learning.SPARSE_VIEWS
    plans = {}
    for nv, sel in ((learning.SPARSE_VIEWS, slice(0, None, step)), (learning.DENSE_VIEWS, slice(None))):
        plans[nv] = (tomo.Plan(tomo.Params(n_vox=n, n_angles=nv, voxel_size=base.voxel, wavelength=base.wavelength,
                                           sigma=base.sigma, epsilon=base.epsilon, n_pix=base.M, n_planes=base.K),
                               dirs[sel], dist[sel], stream=stream), sel)
    total = n_train + n_held
    vols = torch.empty((total, 2, n, n, n), dtype=torch.float32, device=dev)
    t0 = time.time()
    for k in range(total):
        # training phantoms 0 .. 1999; the held-out ones always 2000 .. 2199
        idx = k if k < n_train else learning.TRAIN + (k - n_train)
        ph = learning.pair_phantom(idx, n, base.voxel)
        imgs = learning.born_images_batched(ph, dirs, base.M, base.voxel, base.wavelength, dist, base.sigma)
        for j, nv in enumerate((learning.SPARSE_VIEWS, learning.DENSE_VIEWS)):
            plan, sel = plans[nv]
            plan.reconstruct_async(imgs[sel].contiguous(), vols[k, j], stream=stream)
        if (k + 1) % 100 == 0 or k + 1 == total:
            for plan, _ in plans.values():
                plan.sync(stream)
            print(f"[bench] unet_pairs: {k + 1}/{total} pairs in {time.time() - t0:.0f}s", file=sys.stderr, flush=True)
    gen_s = time.time() - t0
    scale = float(torch.sqrt((vols[:n_train, 1] ** 2).mean()))
    vols /= scale
    net = unet.Net(n)
    theta = torch.from_numpy(netinit.init_params(9)).to(dev)
    m, v, g = torch.zeros_like(theta), torch.zeros_like(theta), torch.empty_like(theta)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    y = torch.empty((n, n, n), device=dev)

    def held_out_mse():
        base_e = corr_e = 0.0
        for k in range(n_train, total):
            net.forward(theta, vols[k, 0], y)
            base_e += float(((vols[k, 0] - vols[k, 1]) ** 2).mean())
            corr_e += float(((y - vols[k, 1]) ** 2).mean())
        return base_e / n_held, corr_e / n_held

    rng = np.random.default_rng(learning.PAIR_SEED)
    steps_total = args.epochs * n_train
    it = 0
    t0 = time.time()
    train_s = 0.0
    for ep in range(args.epochs):
        order = rng.permutation(n_train)
        torch.cuda.synchronize()
        te = time.perf_counter()
        for k in order:
            it += 1
            frac = it / steps_total
            lr = 1e-3 if frac <= 0.5 else 1e-4 + 0.5 * (1e-3 - 1e-4) * (1.0 + np.cos(np.pi * (frac - 0.5) / 0.5))
            net.gradient(theta, vols[k, 0], vols[k, 1], g, loss)
            net.adam(theta, g, m, v, it, float(lr))
        torch.cuda.synchronize()
        train_s += time.perf_counter() - te
        b_e, c_e = held_out_mse()
        print(f"[bench] unet_pairs: epoch {ep + 1}/{args.epochs}: loss {float(loss):.4g}, held-out MSE sparse "
              f"{b_e:.4g} network {c_e:.4g} (ratio {c_e / b_e:.3f}), {time.time() - t0:.0f}s",
              file=sys.stderr, flush=True)
    b_e, c_e = held_out_mse()
    ratio = c_e / b_e
    ms = train_s * 1e3 / steps_total
    out = {
        "metric": "held-out MSE vs the dense reconstruction: network output / plain sparse reconstruction",
        "method": "unet_pairs",
        "value": ratio,
        "unit": "ratio",
        "n_gpus": 1, "steps": steps_total, "warmup": 0, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 weights, f32 activations and sums", "data": "synthetic",
        "config": {"workload": "unet_pairs", "n_vox": n, "train_pairs": n_train, "held_out_pairs": n_held,
                   "sparse_views": learning.SPARSE_VIEWS, "dense_views": learning.DENSE_VIEWS,
                   "epochs": args.epochs, "pair_generation_s": round(gen_s, 1),
                   "training_s": round(train_s, 1), "training_voxels_per_s": n ** 3 / (ms * 1e-3)},
        "held_out": {"mse_sparse_vs_dense": b_e, "mse_network_vs_dense": c_e, "ratio": ratio,
                     "fallback_to_plain_reconstruction": bool(ratio >= 1.0)},
    }
    print(json.dumps(out), flush=True)
    net.destroy()
    for plan, _ in plans.values():
        plan.destroy()


if __name__ == "__main__":
    main()
