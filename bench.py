#!/usr/bin/env python3
"""Throughput of the multislice reconstruction step on one MI355X.

A step is one mini-batch update of the whole hot path through the C ABI
(ptyr_step): sub-pixel probe shift, object transmission and tilted Fresnel
propagation through every slice, far-field intensity summed over modes, the
amplitude (Gaussian, p = 0.5) loss, the gradient with respect to object
amplitude and phase, probe, positions, tilts and slice spacing (object
gradient reduced per tile), and a dense Adam update of all six parameters.

Workload (seeded, synthetic): detector / probe window 128 x 128 at 0.15 A/px,
300 kV, 6 orthogonalised Hermite-Gaussian probe modes, object 12 slices of
640 x 640 (square Gaussian-atom lattice, 5 % vacancies, dz = 20 A), a
128 x 128 raster (step 4 px, +-0.5 px jitter), Poisson data at 1e6
electrons per pattern, 64 positions per update.  All inputs are resident in
device memory before the timed region.

Prints one JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.

`--learned-init` measures the second metric instead: wall time for the
gradient reconstruction of a held-out single-slice object (64 x 64 patterns,
10 x 10 scan, 1e5 electrons per pattern) to reach 0.02 rad RMS phase error
from the learned initial guess, next to the same from the plain initial
object.  The conv net is first trained on 200k neighbourhoods (3,125 random
objects) simulated by the library's forward model; the training and data
times are reported, not counted.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3          # MI355X: 256 CU x 2.4 GHz x 128 FP32 FMA/clk x 2
PEAK_FP32_UNPACKED_TFLOPS = 78.6         # the same without packed FP32 (disabled in this build)
PEAK_HBM_GBS = 8000.0                    # MI355X HBM3E
WORKLOAD = "multislice_128"


def fft_flops(N):
    """Nominal flops of one N x N complex 2-D FFT: 5 N^2 log2(N^2)."""
    import math
    return 5.0 * N * N * math.log2(N * N)


def line_pass_bytes(w, B, n_obj=1):
    """Algorithmic HBM bytes per step of the N=256 line passes (one wave =
    N*N complex64).  Forward, per chain: shifted probe (read the spectrum,
    write Z_0, the wave entering slice 0's row pass) 2 waves; per slice a row
    pass (read Z_s, write the wave) and a column pass (read the wave, write
    the kept Z_{s+1}) 4 waves, the last column pass writing the far field and
    the mode intensity instead (2.5); so 4S + 2.5 waves.  Gradient, per chain:
    6S + 1.5 waves (the column pass also reads Z_s to rebuild Y_s, the row
    pass reads Z_s to rebuild phi_s), plus the patch gradients, which the
    row pass sums over groups of mg probe modes (mg = the largest divisor of
    the probe modes up to 8) and writes once per group: S / mg waves per
    chain.  Object patches are read once per batch row, slice and
    object mode; with n_obj object modes every probe mode meets every object
    mode."""
    wave = w.N * w.N * 8
    chains = B * w.M * n_obj
    patches = B * w.S * wave * n_obj
    mg = max(d for d in range(1, 9) if w.M % d == 0)
    return {"forward": chains * (4 * w.S + 2.5) * wave + patches,
            "gradient": chains * (6 * w.S + w.S / mg + 1.5) * wave + patches}


def copy_calibration(out, dev):
    """Copy a 512 MiB buffer 4 times after one untimed copy: a kernel of known
    size for the HBM counters, and the rate a plain device copy reaches
    (read + write bytes over the event-timed copies)."""
    import torch
    src = torch.ones(128 << 20, dtype=torch.float32, device=dev)     # 512 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(4):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    out["copy_calibration_bytes"] = src.numel() * 4
    out["copy_gbs"] = round(4 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)


def read_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    from paper_2505_07814_amd.profile_summary import source_hash
    if vals.get("source_hash") != source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_activity(kernel, workload):
    """VALU / LDS busy fractions of a kernel from a committed rocprofv3 counter
    summary taken on the current kernel sources ({} if none)."""
    path = os.path.join(ROOT, "profiles", f"activity_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    from paper_2505_07814_amd.profile_summary import source_hash
    if vals.get("source_hash") != source_hash():
        return {}
    out = {}
    for k in ("valu_busy", "lds_busy", "lds_bank_conflict"):
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return out


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo (None if unreadable)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_batch(w, nb, B, amp0, ph0):
    """Measured patterns of batch nb (untimed), then the timed oracle work of
    one step: forward, loss, gradient of all six parameters and Adam."""
    import numpy as np
    from oracle import multislice as ms
    from oracle.adam import adam_step
    from paper_2505_07814_amd import synth

    lam = synth.wavelength_A(w.kv)
    z = np.zeros
    sl = slice(nb * B, (nb + 1) * B)
    pos, tilt = w.pos[sl], w.tilt[sl]
    # measured patterns for the sample come from the oracle itself (untimed)
    I = ms.forward(w.amp, w.phase, w.probe, pos, tilt, w.dz, w.dx, lam)
    meas = synth.poisson(I, w.seed_base + 4 + nb).astype(np.float64)

    def work():
        t0 = time.perf_counter()
        g = ms.gradients(amp0, ph0, w.probe, pos, tilt, w.dz, w.dx, lam, meas)
        adam_step(amp0, g.amp, z(amp0.shape), z(amp0.shape), 0, 1e-3)
        adam_step(ph0, g.phase, z(ph0.shape), z(ph0.shape), 0, 1e-3)
        adam_step(w.probe, g.probe, z(w.probe.shape, complex), z(w.probe.shape, complex), 0, 1e-3)
        adam_step(pos, g.pos, z(pos.shape), z(pos.shape), 0, 1e-3)
        adam_step(tilt, g.tilt, z(tilt.shape), z(tilt.shape), 0, 1e-3)
        return t0, time.perf_counter()
    return work


def _oracle_worker(workload, positions, nb, B, barrier, queue):
    """One all-core worker (a fresh interpreter): its own batch of the
    workload, started together with the others."""
    import numpy as np  # noqa: F401
    from paper_2505_07814_amd import synth
    w = synth.workload(workload, scan=positions or None)
    amp0, ph0 = synth.plain_init(w.S, w.H, w.W, w.seed_base + 5)
    work = _oracle_batch(w, nb, B, amp0, ph0)
    barrier.wait()
    queue.put(work())


def cpu_baseline(w, B, workload, positions, min_seconds=10.0, max_batches=8, max_workers=16):
    """The FP64 oracle on consecutive batches of the same workload (forward,
    loss, gradient of all six parameters and the Adam update, on the host):
    on one thread until at least min_seconds of timed work, then one batch
    per core on every core this process may run on (capped at max_workers),
    started together, timed from the first start to the last finish."""
    from paper_2505_07814_amd import synth

    amp0, ph0 = synth.plain_init(w.S, w.H, w.W, w.seed_base + 5)
    dt, nb = 0.0, 0
    while nb < max_batches and (nb == 0 or dt < min_seconds) and (nb + 1) * B <= w.pos.shape[0]:
        t0, t1 = _oracle_batch(w, nb, B, amp0, ph0)()
        dt += t1 - t0
        nb += 1
    out = {"value": nb * B / dt, "unit": "patterns/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{nb} batches of {B} positions of the same workload (forward, loss, gradient of all six "
                     f"parameters and Adam, FP64 NumPy with the oracle's own radix-2 FFT, single thread), "
                     f"{dt:.1f} s timed"}
    cores = len(os.sched_getaffinity(0))
    n = min(cores, max_workers, w.pos.shape[0] // B)
    if n > 1:
        import multiprocessing as mp
        ctx = mp.get_context("spawn")                  # fresh interpreters: nothing of the GPU runtime
        barrier, queue = ctx.Barrier(n), ctx.Queue()
        procs = [ctx.Process(target=_oracle_worker, args=(workload, positions, k, B, barrier, queue))
                 for k in range(n)]
        for p in procs:
            p.start()
        spans = [queue.get() for _ in range(n)]
        for p in procs:
            p.join()
        wall = max(t1 for _, t1 in spans) - min(t0 for t0, _ in spans)
        out["all_cores"] = {"value": n * B / wall, "unit": "patterns/s", "cores": n,
                            "sample": f"{n} batches of {B} positions, one per process (NumPy single-threaded in "
                                      f"each), {wall:.1f} s from the first start to the last finish; "
                                      f"{cores} cores available to this process"}
    return out


def learned_init_run(objects, epochs, iterations, dev):
    """Train the conv net on `objects` simulated objects (64 neighbourhoods
    each), then reconstruct the held-out object from the learned and from the
    plain initial guess: (learned result, plain result, training result,
    inference seconds, number of pairs, data seconds)."""
    import numpy as np
    import torch

    from paper_2505_07814_amd import learned_init as li
    from paper_2505_07814_amd import synth
    from paper_2505_07814_amd.cnn import ConvInit

    log = lambda m: print(m, file=sys.stderr, flush=True)
    data = li.make_dataset(objects, dev)
    data_s, n_pairs = data.seconds, data.nbr.shape[0]
    log(f"data: {n_pairs} pairs from {objects} objects in {data_s:.1f} s")
    net = ConvInit(256, device=dev)
    res = li.train(data, epochs=epochs, batch=256, lr=1e-3, net=net, log=log)
    del data
    case = li.eval_case(dev)
    plain = torch.from_numpy(synth.plain_init(1, synth.LI_H, synth.LI_H, 5)[1][0].astype(np.float32)).to(dev)
    li.learned_phase(net, res.params, case, plain)          # warm-up of the inference launches
    li.reconstruct(case, plain, 2)                           # and of the reconstruction launches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    init = li.learned_phase(net, res.params, case, plain)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    r_plain = li.reconstruct(case, plain, iterations)
    r_learn = li.reconstruct(case, init, iterations, setup_seconds=setup)
    return r_learn, r_plain, res, setup, n_pairs, data_s


def learned_init_block(objects, epochs, iterations, dev, errors=False):
    """Metric 2 as a JSON object: iterations and wall seconds to 0.02 rad RMS
    phase error from either start, and the (uncounted) training time."""
    r_learn, r_plain, res, setup, n_pairs, data_s = learned_init_run(objects, epochs, iterations, dev)
    rnd = lambda x: None if x is None else round(x, 5)
    blk = {
        "target_rad": 0.02,
        "learned_init": {"iterations": r_learn.iterations_to_target, "seconds": rnd(r_learn.seconds_to_target),
                         "inference_seconds": round(setup, 5)},
        "plain_init": {"iterations": r_plain.iterations_to_target, "seconds": rnd(r_plain.seconds_to_target)},
        "training": {"seconds": round(res.seconds, 2), "data_seconds": round(data_s, 2), "pairs": int(n_pairs),
                     "objects": objects, "epochs": epochs},
        "note": "held-out single-slice object (seed 999), 64 x 64 patterns, 10 x 10 scan, Adam lr 1e-2 on "
                "amplitude and phase, 20 positions per step; seconds include the net's inference and stitching "
                "for the learned start; training and data simulation are reported, not counted",
    }
    if errors:
        blk["learned_init"]["errors"] = [round(e, 5) for e in r_learn.errors]
        blk["plain_init"]["errors"] = [round(e, 5) for e in r_plain.errors]
        blk["training"]["epoch_losses"] = [float(f"{x:.4e}") for x in res.losses]
    return blk


def learned_init_bench(args):
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    blk = learned_init_block(args.objects, args.epochs, args.iterations, dev, errors=True)
    out = {
        "metric": "wall time to 0.02 rad RMS phase error (learned init + hand adjoint)",
        "value": blk["learned_init"]["seconds"],
        "unit": "s", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
        "dtype": "bf16 net / f32 reconstruction", "data": "synthetic",
        "config": {"workload": "single-slice 64x64 at 0.2 A/px, 300 kV, 20 mrad, 100 A defocus, 1e5 e/pattern; "
                               "objects 144x144 with 51 random Gaussian atoms (0.5 rad); 10x10 raster, step 8 px; "
                               "eval object seed 999; reconstruction: Adam lr 1e-2 on amplitude and phase, "
                               "20 positions per step, Gaussian amplitude loss",
                   "train_pairs": blk["training"]["pairs"], "train_objects": args.objects,
                   "epochs": args.epochs},
        **{k: blk[k] for k in ("learned_init", "plain_init", "training")},
    }
    print(json.dumps(out), flush=True)


def sweep_bench(args):
    """Throughput of the full step around the N=128 point, one axis at a
    time: batch B, probe modes M (the first M of the six), slices S (the
    first S of the twelve, or the twelve twice for 24).  Timing only: the
    measured patterns are those of the 12-slice, 6-mode object for every
    shape."""
    import numpy as np
    import torch

    from paper_2505_07814_amd import synth
    from paper_2505_07814_amd.ptyr import AdamState, Engine

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.workload("multislice_128", scan=8192)
    lam = synth.wavelength_A(w.kv)
    n_pos = w.pos.shape[0]
    T = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a if dt is None else a.astype(dt))).to(dev)
    meas = torch.poisson(torch.full((n_pos, w.N, w.N), 60.0, device=dev))
    amp0, ph0 = synth.plain_init(w.S, w.H, w.W, w.seed_base + 5)
    lr = dict(amp=5e-4, phase=5e-4, probe=1e-4, pos=1e-3, tilt=1e-5, dz=1e-2)
    points = [(64, 6, 12)] + [(b, 6, 12) for b in (16, 32, 128, 256)] + [(64, m, 12) for m in (1, 3)] + \
             [(64, 6, s) for s in (1, 6, 24)]
    rows = []
    for B, M, S in points:
        reps = (S + 11) // 12
        amp = np.concatenate([amp0] * reps)[:S]
        ph = np.concatenate([ph0] * reps)[:S]
        eng = Engine(w.N, M, S, w.H, w.W, B, w.dx, lam, n_scan=n_pos, device=dev)
        st = AdamState(T(amp, np.float32), T(ph, np.float32), T(w.probe[:M], np.complex64), T(w.pos, np.float32),
                       T(np.zeros_like(w.pos), np.float32), T(np.array([w.dz], np.float32)))
        perm = np.random.default_rng(7).permutation(n_pos)
        batches = [torch.tensor(perm[i * B:(i + 1) * B], dtype=torch.int32, device=dev) for i in range(n_pos // B)]
        steps = max(8, min(64, 4096 // B))
        for i in range(4):
            eng.step(st, batches[i % len(batches)], meas, lr)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(steps):
            eng.step(st, batches[(4 + i) % len(batches)], meas, lr)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        rows.append({"B": B, "M": M, "S": S, "ms_per_step": round(ms, 4), "patterns_per_s": round(B / ms * 1e3, 1),
                     "chain_slices_per_s": round(B * M * S / ms * 1e3, 1)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        del eng, st
    print(json.dumps({"metric": "fwd+adjoint patterns/s sweep around N=128, 12 slices, 6 modes, B=64",
                      "unit": "patterns/s", "n_gpus": 1, "data": "synthetic (timing only)", "rows": rows}), flush=True)


def constraints_bench(args):
    """Per-iteration constraints (ptyr_constrain) on the N=128 workload's
    object and probe: r_z depth filter (sigma = 1 slice) of amplitude and
    phase, phase positivity, orthogonalisation of the six probe modes.  The
    dominant kernel is the depth filter, bound by HBM: one launch reads and
    writes both 12 x 640 x 640 float fields.  The k_z filter is timed on its
    own and reported beside it."""
    import numpy as np
    import torch

    from paper_2505_07814_amd import synth
    from paper_2505_07814_amd.ptyr import Engine

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.workload("multislice_128", scan=64)
    lam = synth.wavelength_A(w.kv)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).to(dev)
    amp, ph = T(w.amp, np.float32), T(w.phase - 0.05, np.float32)
    probe = T(w.probe, np.complex64)
    eng = Engine(w.N, w.M, w.S, w.H, w.W, 1, w.dx, lam, device=dev)
    cfg = dict(rz_sigma=1.0, phase_positive=True, probe_orthogonal=True)
    for _ in range(args.warmup):
        eng.constrain(amp, ph, probe, **cfg)
    eng.sync()
    eng.timing(True)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        eng.constrain(amp, ph, probe, **cfg)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_call = e0.elapsed_time(e1) / args.steps
    kt = eng.timing_read()
    eng.timing(False)
    rz_ms, rz_n = kt["rz"]
    launch_bytes = 2 * 2 * w.S * w.H * w.W * 4            # amplitude and phase, each read and written
    achieved = launch_bytes * rz_n / (rz_ms * 1e-3) / 1e9
    out = {"metric": "ptyr_constrain calls/s (N=128 workload: 12 x 640 x 640 object, 6 probe modes)",
           "value": round(1e3 / ms_call, 1), "unit": "calls/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_call": round(ms_call, 4), "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "constraints on multislice_128: r_z filter sigma 1 slice on amplitude and phase, "
                                  "phase positivity, orthogonalisation of 6 probe modes of 128 x 128"},
           "roofline": {"bound": "hbm", "kernel": "k_rz_filter_reg4", "achieved": round(achieved, 1),
                        "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                        "traffic": None, "launch_ms": round(rz_ms / rz_n, 4), "bytes_per_launch": launch_bytes}}
    if not args.no_cpu_baseline:
        from oracle import constraints as oc
        t0 = time.perf_counter()
        oc.apply(w.amp, w.phase, w.probe, **cfg)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(1.0 / dt, 3), "unit": "calls/s", "cores": 1, "kind": "oracle",
                               "sample": "one call on the full object and probe (numpy, float64)"}
    out["roofline"]["traffic"] = read_traffic("rz", "constraints_128")
    # k_z filter (beta 0.1, alpha 1 A^2) alone: amplitude + i phase through
    # five line passes (forward x, forward y, z forward + weight + inverse,
    # inverse y, inverse x), each reading and writing 8 bytes per voxel
    kz = dict(kz_beta=0.1, kz_alpha=1.0, kz_dz=float(w.dz))
    for _ in range(4):
        eng.constrain(amp, ph, **kz)
    torch.cuda.synchronize()
    n_kz = max(8, args.steps // 8)
    e0.record(stream)
    for _ in range(n_kz):
        eng.constrain(amp, ph, **kz)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_kz = e0.elapsed_time(e1) / n_kz

    passes = 5
    kz_bytes = 16 * passes * w.S * w.H * w.W
    out["kz_filter"] = {"ms_per_call": round(ms_kz, 4), "passes": passes, "bytes_per_call": kz_bytes,
                        "achieved_GBs": round(kz_bytes / (ms_kz * 1e-3) / 1e9, 1),
                        "frac_of_hbm_peak": round(kz_bytes / (ms_kz * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                        "traffic": read_traffic("kz", "constraints_128")}
    if args.copy_calibration:
        copy_calibration(out, dev)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=256, help="timed steps (256 = one pass over the scan)")
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--prewarm", type=float, default=1.0,
                    help="seconds of untimed steps before the warmup steps (0: none)")
    ap.add_argument("--batch", type=int, default=0, help="positions per step (0 = the workload's: 64, or 16 at N=256)")
    ap.add_argument("--workload", default=WORKLOAD, choices=["multislice_128", "large_256"],
                    help="multislice_128 is the headline configuration; large_256 measures the N=256 line passes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned-init", action="store_true",
                    help="leave the learned-init block (metric 2) out of the default line")
    ap.add_argument("--positions", type=int, default=0,
                    help="use only the first P scan positions (profiling runs; 0 = all)")
    ap.add_argument("--sweep", action="store_true", help="time the step over B, M and S around the N=128 point")
    ap.add_argument("--learned-init", action="store_true",
                    help="measure wall time to 0.02 rad RMS phase error, learned vs plain initial guess")
    ap.add_argument("--objects", type=int, default=3125, help="training objects for --learned-init (64 pairs each)")
    ap.add_argument("--epochs", type=int, default=16, help="training epochs for --learned-init")
    ap.add_argument("--iterations", type=int, default=60, help="reconstruction iterations for --learned-init")
    ap.add_argument("--sparse-w", type=float, default=0.0,
                    help="weight of the L1 sparsity term of the object phase in the step's loss (0 = off)")
    ap.add_argument("--pacbed-w", type=float, default=0.0,
                    help="weight of the PACBED term in the step's loss (0 = off; on, a batch runs on one stream)")
    ap.add_argument("--obj-modes", type=int, default=1,
                    help="object modes (the extra modes are weaker, partly different copies of the object)")
    ap.add_argument("--constraints", action="store_true",
                    help="time ptyr_constrain (r_z filter, positivity, probe orthogonalisation) on the N=128 workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, copy a 512 MiB buffer 4 times (known-size kernel for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on a single GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.learned_init:
        return learned_init_bench(args)
    if args.sweep:
        return sweep_bench(args)
    if args.constraints:
        return constraints_bench(args)

    import numpy as np
    import torch

    from paper_2505_07814_amd import synth
    from paper_2505_07814_amd.ptyr import AdamState, Engine

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    workload = args.workload
    w = synth.workload(workload, scan=args.positions or None)
    B = args.batch or w.B
    lam = synth.wavelength_A(w.kv)
    n_pos = w.pos.shape[0]
    T = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a if dt is None else a.astype(dt))).to(dev)

    K = args.obj_modes
    eng = Engine(w.N, w.M, w.S, w.H, w.W, B, w.dx, lam, n_scan=n_pos, sparse_w=args.sparse_w,
                 pacbed_w=args.pacbed_w, n_obj=K, device=dev)
    obj = lambda x, f: x if K == 1 else np.stack([x * f ** k for k in range(K)])
    # synthetic measured data: forward model of the true object, Poisson-sampled
    true = dict(amp=T(obj(w.amp, 0.9), np.float32), phase=T(obj(w.phase, 0.7), np.float32),
                probe=T(w.probe, np.complex64),
                pos=T(w.pos, np.float32), tilt=T(w.tilt, np.float32), dz=T(np.array([w.dz], np.float32)))
    meas = torch.empty((n_pos, w.N, w.N), dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(w.seed_base + 4)
    for b0 in range(0, n_pos, B):
        idx = torch.arange(b0, min(b0 + B, n_pos), dtype=torch.int32, device=dev)
        I = eng.forward(true["amp"], true["phase"], true["probe"], true["pos"], true["tilt"], true["dz"], idx=idx)
        meas[b0:b0 + len(idx)] = torch.poisson(I, generator=gen)
    eng.sync()
    del true

    amp0, ph0 = synth.plain_init(w.S, w.H, w.W, w.seed_base + 5)
    st = AdamState(T(obj(amp0, 1.0), np.float32), T(obj(ph0, 1.0), np.float32), T(w.probe, np.complex64),
                   T(w.pos, np.float32),
                   T(np.zeros_like(w.pos), np.float32), T(np.array([w.dz], np.float32)))
    lr = dict(amp=5e-4, phase=5e-4, probe=1e-4, pos=1e-3, tilt=1e-5, dz=1e-2)
    perm = np.random.default_rng(w.seed_base + 6).permutation(n_pos)
    nb = n_pos // B
    batches = [torch.tensor(perm[b * B:(b + 1) * B], dtype=torch.int32, device=dev) for b in range(nb)]

    stream = torch.cuda.current_stream(dev)
    # Before the W warmup steps the step runs untimed for args.prewarm seconds
    # of wall time: a process started right after another GPU process has
    # been seen to run its first few hundred milliseconds of steps 10-15 %
    # slower (later windows of the same process, and its kernels, were not),
    # which a 5-step warmup and a 20-step timed window would measure.
    n_pre, t_pre = 0, time.perf_counter()
    while time.perf_counter() - t_pre < args.prewarm:
        for _ in range(8):
            eng.step(st, batches[n_pre % nb], meas, lr)
            n_pre += 1
        torch.cuda.synchronize()
    t_pre = time.perf_counter() - t_pre
    for s in range(args.warmup):
        eng.step(st, batches[s % nb], meas, lr)
    eng.sync()
    eng.timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for s in range(args.steps):
        eng.step(st, batches[(args.warmup + s) % nb], meas, lr)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    kt = eng.timing_read()
    eng.timing(False)
    eng.sync()
    # the same batches through ptyr_adjoint alone (forward, loss and the six
    # gradients, no Adam), reported beside the step
    grads = {k: torch.zeros_like(getattr(st, k)) for k in st.NAMES}
    params = [getattr(st, k) for k in st.NAMES]
    for s in range(min(args.warmup, 4)):
        eng.adjoint(*params, meas, idx=batches[s % nb], grads=grads)
    torch.cuda.synchronize()
    n_adj = min(args.steps, 16)
    e0.record(stream)
    for s in range(n_adj):
        eng.adjoint(*params, meas, idx=batches[(args.warmup + s) % nb], grads=grads)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_adj = e0.elapsed_time(e1) / n_adj
    eng.sync()

    ms_step = ms_total / args.steps
    value = B * args.steps / (ms_total / 1e3)
    # A batch whose chains exceed one round of workgroups runs as two row
    # ranges on two streams, so each fused kernel has two launches of
    # different sizes per step: flops and durations are summed over all
    # launches.  Concurrent launches share the chip, so the sum of their
    # durations overstates the time each used and `achieved` is a lower bound.
    per_launch = {k: (v[0] / v[1] if v[1] else float("nan")) for k, v in kt.items()}
    dom = max(per_launch, key=lambda k: kt[k][0])
    launches = kt[dom][1]
    if w.N < 256:
        # wave-resident chains: bound by the FFT arithmetic
        flops_step = B * w.M * K * 2 * w.S * fft_flops(w.N)   # nominal FFT flops of either fused kernel per step
        achieved = flops_step * args.steps / (kt[dom][0] * 1e-3) / 1e12
        roofline = {
            "bound": "alu", "kernel": f"k_{dom}<{w.N}>", "achieved": round(achieved, 3),
            "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
            "traffic": read_traffic(dom, workload) if K == 1 else None,
            **(read_activity(dom, workload) if K == 1 else {}),
            "launch_ms": round(per_launch[dom], 4),
            "launches_per_step": launches / args.steps,
            "flops_per_launch": flops_step * args.steps / launches,
            "peak_without_packed_fp32": PEAK_FP32_UNPACKED_TFLOPS,
            "other_kernel_ms": {k: round(v, 4) for k, v in per_launch.items() if k != dom},
        }
    else:
        # line passes: every pass reads and writes the chain's wave through HBM
        by = line_pass_bytes(w, B, K)[dom]
        achieved = by * args.steps / (kt[dom][0] * 1e-3) / 1e9
        roofline = {
            "bound": "hbm", "kernel": f"{dom} line passes (N=256)", "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": read_traffic(dom, workload) if K == 1 else None,
            "launch_ms": round(per_launch[dom], 4),
            "launches_per_step": launches / args.steps,
            "bytes_per_launch": by * args.steps / launches,
            "other_kernel_ms": {k: round(v, 4) for k, v in per_launch.items() if k != dom},
        }
    desc = {
        "multislice_128": "multislice_128: probe 128x128 at 0.15 A/px, 6 modes, object 12 x 640 x 640, dz 20 A, "
                          "128x128 scan, 64 positions per Adam step (forward + loss + gradient of all six "
                          "parameters + Adam)",
        "large_256": "large_256: probe 256x256 at 0.15 A/px, 8 modes, object 30 x 1024 x 1024 (twisted hexagonal "
                     "bilayer), dz 10 A, 192x192 scan, 16 positions per Adam step (forward + loss + gradient of "
                     "all six parameters + Adam)",
    }[workload]
    metric = ("fwd+adjoint patterns/s (N=128, 12 slices, 6 modes)" if workload == "multislice_128"
              else "fwd+adjoint patterns/s (N=256, 30 slices, 8 modes)")
    out = {
        "metric": metric,
        "value": round(value, 1), "unit": "patterns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "prewarm": {"seconds": round(t_pre, 3), "steps": n_pre},
        "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "global_batch": B, "N": w.N, "slices": w.S, "modes": w.M, "positions": n_pos,
                   **({"sparse_w": args.sparse_w} if args.sparse_w else {}),
                   **({"pacbed_w": args.pacbed_w} if args.pacbed_w else {}),
                   **({"object_modes": K} if K > 1 else {})},
        "roofline": roofline,
        "fwd_adjoint_only": {"ms_per_step": round(ms_adj, 4), "value": round(B / (ms_adj * 1e-3), 1),
                             "unit": "patterns/s", "steps": n_adj,
                             "note": "ptyr_adjoint on the first batches of the timed ones: forward, loss, all six "
                                     "gradients, no Adam"},
    }
    if not args.no_learned_init and workload == "multislice_128" and K == 1:
        del st, eng, meas, batches, grads, params
        torch.cuda.empty_cache()
        out["learned_init"] = learned_init_block(args.objects, args.epochs, args.iterations, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, B, workload, args.positions)
    if args.copy_calibration:
        copy_calibration(out, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
