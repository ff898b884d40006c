"""Benchmark: discrete-gradient step of Discrete Morse Sandwich on one MI355X.

One step = global vertex order (dms_order) + ProcessLowerStars gradient
(dms_discrete_gradient) + critical-simplex extraction (dms_critical_simplices)
over the workload below, with the input field already resident in HBM.

Workload (default): a 1026^3 float32 block with a one-voxel ghost layer --
512 isotropic Gaussians (seed 3) plus 1e-3 uniform noise -- whose owned
1024^3 interior is processed: one GPU's share of a distributed run at its real
shape.  Throughput = owned vertices per second.

Printed: one JSON line with the metric, per-stage times (HIP events on the
stream the kernels run on), the roofline object of the dominant kernel and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# algorithmic bytes per owned vertex of each stage (what the method must move)
# (gradient: order read + record write + critical-mask bit; critical: see MASK_BYTES)
MASK_BYTES = 1.0 / 8.0
ALG_BYTES = {"order": 8.0, "gradient": 20.0 + MASK_BYTES, "critical": 16.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--owned", type=int, default=1024, help="owned vertices per side")
    ap.add_argument("--bumps", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and differentiable lines")
    ap.add_argument("--cpu-planes", type=int, default=48, help="owned z-planes in the oracle sample")
    ap.add_argument("--large", action="store_true",
                    help="time the order-free path (gradient from the values + extraction) on the "
                         "2048x1920x1536 float32 field instead (one JSON line of its own)")
    ap.add_argument("--only", choices=["batched", "differentiable", "small"], default=None,
                    help="run only the batched (96-field), the differentiable (128^3 f64) or the "
                         "64^3 and 512^3 part and print its object as the JSON line")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    return ap.parse_args()


def copy_bandwidth(dev, mib=4096, reps=5):
    """Measured streaming bandwidth of a plain device-to-device copy (read +
    write bytes / time, GB/s), reported next to the 8 TB/s spec peak."""
    import torch
    src = torch.empty(mib << 18, dtype=torch.int32, device=dev).fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * mib * (1 << 20) / (ms / 1e3) / 1e9, 1)


def measured_traffic_gb():
    """HBM bytes per gradient call (GB) from the committed counter summary,
    or None when the kernel source has changed since the counters were taken."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_2505_21266_amd", "csrc", "dms_gradient.hip")
    prof = os.path.join(ROOT, "profiles", "traffic_k_gradient_gauss1026.md")
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        m = re.search(r"traffic: kernel=dms_discrete_gradient source_sha256=([0-9a-f]+) "
                      r"bytes_per_call=(\d+)", open(prof).read())
    except OSError:
        return None
    if not m or m.group(1) != sha:
        return None
    return round(int(m.group(2)) / 1e9, 2)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_stages(sub, lo, hi, threads):
    """Order, ProcessLowerStars and extraction of box [lo, hi) of the slab sub
    with the CPU oracle on `threads` threads; returns (owned vertices, seconds
    per stage)."""
    import oracle
    nz, ny, nx = sub.shape
    dims = (nx, ny, nz)
    t0 = time.perf_counter()
    o = oracle.order(sub, nthreads=threads)
    t1 = time.perf_counter()
    rec, counts, an = oracle.lower_stars(o, dims, lo, hi, nthreads=threads)
    t2 = time.perf_counter()
    oracle.critical_simplices(rec, dims, lo, hi, nthreads=threads)
    t3 = time.perf_counter()
    owned = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2])
    return owned, (t1 - t0, t2 - t1, t3 - t2)


def cpu_baseline(field, lo, hi, planes):
    """Times the CPU oracle (order, ProcessLowerStars, extraction) on a slab of
    the same field -- `planes` owned z-planes plus their ghost planes -- on
    every host core the process may use, each stage threaded (the sort as
    sorted runs merged pairwise, the lower stars and the extraction over rows).
    Beside it, one thread on the 64^3 noise workload and on a 16-plane slab of
    the 512^3 Gaussian one."""
    from paper_2505_21266_amd import inputs
    k0 = lo[2]
    sub = np.ascontiguousarray(field[k0 - 1:k0 + planes + 1])
    threads = len(os.sched_getaffinity(0))
    owned, (t_o, t_s, t_c) = _oracle_stages(sub, (lo[0], lo[1], 1), (hi[0], hi[1], 1 + planes), threads)
    one = {}
    v1 = inputs.config1()
    n1, st1 = _oracle_stages(v1, (0, 0, 0), (64, 64, 64), 1)
    one["noise64"] = round(n1 / sum(st1) / 1e9, 6)
    v2 = inputs.config2()[:18]  # owned planes 1..16 of the 512^3 field, with their neighbours
    n2, st2 = _oracle_stages(np.ascontiguousarray(v2), (0, 0, 1), (512, 512, 17), 1)
    one["gauss512_16planes"] = round(n2 / sum(st2) / 1e9, 6)
    return {
        "value": owned / (t_o + t_s + t_c) / 1e9,
        "unit": "Gvertices/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d owned z-planes (%dx%dx%d owned vertices, %.1f M) of the same field, %d threads in "
                  "every stage: order %.2f s, lower stars %.2f s, extraction %.2f s; CPU: %s"
                  % (planes, hi[0] - lo[0], hi[1] - lo[1], planes, owned / 1e6, threads, t_o, t_s, t_c,
                     cpu_model()),
        "one_thread_gvertices_per_s": one,
    }


def bench_batched(dev, reps):
    """96 float32 fields with sides U{32..256} per axis (half white noise, half
    16-Gaussian mixtures): one captured graph per batch, timed over replays."""
    import torch

    import paper_2505_21266_amd as dms
    from paper_2505_21266_amd import inputs
    fields, sides = inputs.config4()
    vals = torch.from_numpy(np.concatenate([f.reshape(-1) for f in fields])).to(dev)
    del fields
    b = dms.Batch([tuple(int(x) for x in s) for s in sides], tune=True)
    b.run(vals)  # tunes the tile shape, then captures the graph
    bufs = b.bufs
    for _ in range(2):
        b.launch(vals, bufs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.launch(vals, bufs)
    e1.record()
    torch.cuda.synchronize()
    if int(bufs["flags"].item()) != 0:
        raise RuntimeError("batched run set device flags")
    ms = e0.elapsed_time(e1) / reps
    return {"fields": b.nfields, "vertices": b.total, "ms_per_batch": round(ms, 3),
            "fields_per_s": round(b.nfields / (ms / 1e3), 1),
            "gvertices_per_s": round(b.total / (ms / 1e3) / 1e9, 3),
            "tile_variant": ["64x16", "32x32", "16x64"][b.variant], "replays": reps}


def bench_differentiable(dev, reps):
    """128^3 float64 field (16 Gaussians + 1e-4 noise, min gap 1e-9): GPU
    forward (order, gradient, extraction), D0 pairing (extremum graph on the
    GPU, union-find on the host), GPU backward.  The all-host D0 pairing is
    timed beside it for comparison, and the D2 pairing (ascents on the dual
    complex on the GPU, union-find on the host) after it."""
    import torch

    import paper_2505_21266_amd as dms
    from paper_2505_21266_amd import inputs
    f = inputs.config5()
    x = torch.from_numpy(f).to(dev)
    dims = dms.dims_of(x)
    n = x.numel()
    o = dms.order(x)
    rec = dms.discrete_gradient(o)
    lists, counts = dms.critical_simplices(rec, dims)
    cap = counts.cpu().numpy()
    torch.cuda.synchronize()
    fwd, host, bwd, allhost, d2 = [], [], [], [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        o = dms.order(x, check=False)
        rec = dms.discrete_gradient(o)
        lists, counts = dms.critical_simplices(rec, dims, cap=cap)
        e[1].record()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pe, pm = dms.d0_pairs(rec, o, dims, lists[0], lists[1])
        t1 = time.perf_counter()
        t2 = time.perf_counter()
        pe2, pm2 = dms.d0_pairs_host(rec.cpu().numpy(), o.cpu().numpy().reshape(-1), dims,
                                     lists[1].cpu().numpy())
        allhost.append((time.perf_counter() - t2) * 1e3)
        if not ((pe2 == pe).all() and (pm2 == pm).all()):
            raise RuntimeError("D0 pairings disagree")
        t3 = time.perf_counter()
        pt, pq = dms.d2_pairs(rec, o, dims, lists[2], lists[3])
        d2.append((time.perf_counter() - t3) * 1e3)
        dc = torch.from_numpy(pe).to(dev)
        bc = torch.from_numpy(pm).to(dev) << 8
        flat = x.reshape(-1)
        pers = flat[dc >> 8] - flat[bc >> 8]
        keep = (pers < 0.05).double()
        gd = (2.0 * pers * keep).contiguous()
        gb = (-2.0 * pers * keep).contiguous()
        e[2].record()
        dms.gradient_backward(bc, dc, gb, gd, n)
        e[3].record()
        torch.cuda.synchronize()
        fwd.append(e[0].elapsed_time(e[1]))
        host.append((t1 - t0) * 1e3)
        bwd.append(e[2].elapsed_time(e[3]))
    return {"vertices": n, "pairs": int(pe.size), "forward_gpu_ms": round(float(np.median(fwd)), 3),
            "d0_ms": round(float(np.median(host)), 3),
            "d0_all_host_ms": round(float(np.median(allhost)), 3),
            "d2_pairs": int(pt.size), "d2_ms": round(float(np.median(d2)), 3),
            "backward_gpu_ms": round(float(np.median(bwd)), 4), "reps": reps}


def bench_small_configs(dev, reps):
    """The 64^3 noise and 512^3 Gaussian fields: the step (order, gradient
    with the critical mask, masked extraction) timed per stage with HIP
    events on the stream (median of `reps`), and the CPU oracle on the same
    whole field on every host core."""
    import torch

    import paper_2505_21266_amd as dms
    from paper_2505_21266_amd import inputs
    out = {}
    threads = len(os.sched_getaffinity(0))
    for name, field in (("noise64", inputs.config1()), ("gauss512", inputs.config2())):
        nz, ny, nx = field.shape
        dims = (nx, ny, nz)
        n = nx * ny * nz
        values = torch.from_numpy(field).to(dev)
        order_t = torch.empty(values.shape, dtype=torch.int32, device=dev)
        rec = torch.empty((n, 4), dtype=torch.int32, device=dev)
        mask = dms.critical_mask(n, dev)
        gws = dms.gradient_workspace(order_t)
        flags = dms.new_flags(dev)
        dms.order(values, out=order_t)
        dms.discrete_gradient(order_t, out=rec, workspace=gws, mask=mask)
        lists, counts = dms.critical_simplices(rec, dims, mask=mask)
        cap = counts.cpu().numpy().copy()
        counts_t = torch.zeros(4, dtype=torch.int64, device=dev)
        stream = torch.cuda.current_stream(dev)
        stages = []
        for _ in range(reps + 1):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record(stream)
            dms.order(values, out=order_t, flags=flags, check=False)
            e[1].record(stream)
            dms.discrete_gradient(order_t, out=rec, workspace=gws, mask=mask)
            e[2].record(stream)
            dms.critical_simplices(rec, dims, cap=cap, flags=flags, counts=counts_t, mask=mask)
            e[3].record(stream)
            torch.cuda.synchronize()
            stages.append([e[i].elapsed_time(e[i + 1]) for i in range(3)])
        if int(flags.item()) != 0:
            raise RuntimeError("device flags set: %d" % int(flags.item()))
        med = np.median(np.asarray(stages[1:]), axis=0)
        del values, order_t, rec, mask, gws, lists
        torch.cuda.empty_cache()
        owned, st = _oracle_stages(field, (0, 0, 0), dims, threads)
        out[name] = {"vertices": n, "gpu_ms": {"order": round(float(med[0]), 3),
                                               "gradient": round(float(med[1]), 3),
                                               "critical": round(float(med[2]), 3)},
                     "gvertices_per_s": round(n / (float(med.sum()) / 1e3) / 1e9, 3),
                     "critical_counts": [int(c) for c in cap],
                     "oracle_s": {"order": round(st[0], 3), "lower_stars": round(st[1], 3),
                                  "extraction": round(st[2], 3)},
                     "oracle_threads": threads}
    return out


def bench_large(args, dev):
    """The paper's largest shape, 2048 x 1920 x 1536 float32 (6.04e9
    vertices): beyond int32 orders, so the step is the gradient straight
    from the values plus the extraction."""
    import torch

    import paper_2505_21266_amd as dms
    from paper_2505_21266_amd import inputs
    t0 = time.perf_counter()
    field = inputs.config_large()
    gen_s = time.perf_counter() - t0
    nz, ny, nx = field.shape
    dims = (nx, ny, nz)
    n = nx * ny * nz
    values = torch.from_numpy(field).to(dev)
    del field
    rec = torch.empty((n, 4), dtype=torch.int32, device=dev)
    lo, hi = (0, 0, 0), dims
    gws = torch.empty(int(dms.lib().dms_gradient_workspace_size(dms._arr3(dims)[1], dms._arr3(lo)[1],
                                                                    dms._arr3(hi)[1])),
                      dtype=torch.uint8, device=dev)
    flags = dms.new_flags(dev)
    mask = dms.critical_mask(n, dev)
    dms.discrete_gradient_values(values, out=rec, workspace=gws, flags=flags, check=False, mask=mask)
    lists, counts = dms.critical_simplices(rec, dims, mask=mask)
    cap = counts.cpu().numpy().copy()
    counts_t = torch.zeros(4, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        dms.discrete_gradient_values(values, out=rec, workspace=gws, flags=flags, check=False, mask=mask)
        if ev is not None:
            ev[1].record(stream)
        dms.critical_simplices(rec, dims, cap=cap, flags=flags, counts=counts_t, mask=mask)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t1 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    if int(flags.item()) != 0:
        raise RuntimeError("device flags set: %d" % int(flags.item()))
    grad_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    crit_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms_step = wall / args.steps * 1e3
    out = {
        "metric": "discrete-gradient Gvertices/s from the values (gradient + critical) at 2048x1920x1536 f32",
        "value": round(n / (ms_step / 1e3) / 1e9, 3), "unit": "Gvertices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "mix6g: 2048x1920x1536 float32, 64 Gaussians + 1e-3 U[0,1) noise (seed 6)",
                   "vertices": n, "critical_counts": [int(c) for c in cap]},
        "stage_ms": {"gradient_from_values": round(grad_ms, 3), "critical": round(crit_ms, 3)},
        "input_gen_s": round(gen_s, 1),
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the kernels work on one GPU's block); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2505_21266_amd as dms
    from paper_2505_21266_amd import inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.large:
        bench_large(args, dev)
        return
    if args.only == "batched":
        print(json.dumps(bench_batched(dev, max(args.steps, 3))), flush=True)
        return
    if args.only == "small":
        print(json.dumps(bench_small_configs(dev, max(args.steps, 3))), flush=True)
        return
    if args.only == "differentiable":
        print(json.dumps(bench_differentiable(dev, max(args.steps, 3))), flush=True)
        return
    if args.copy_mib:
        src = torch.ones(args.copy_mib * (1 << 18), dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_gen = time.perf_counter()
    field, lo, hi = inputs.config3(args.owned, args.bumps)
    t_gen = time.perf_counter() - t_gen
    nz, ny, nx = field.shape
    dims = (nx, ny, nz)
    owned = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2])
    values = torch.from_numpy(field).to(dev)

    stream = torch.cuda.current_stream(dev)
    order_t = torch.empty(values.shape, dtype=torch.int32, device=dev)
    rec = torch.empty((owned, 4), dtype=torch.int32, device=dev)
    flags = dms.new_flags(dev)
    gws = dms.gradient_workspace(order_t, lo, hi)
    mask = dms.critical_mask(owned, dev)
    # capacities from one exact run (the counts do not change between steps)
    dms.order(values, out=order_t)
    dms.discrete_gradient(order_t, lo, hi, out=rec, workspace=gws, mask=mask)
    lists, counts = dms.critical_simplices(rec, dims, lo, hi, mask=mask)
    cap = counts.cpu().numpy().copy()
    counts_t = torch.zeros(4, dtype=torch.int64, device=dev)
    flagged = int(np.unpackbits(mask.cpu().numpy().view(np.uint8)).sum())

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        dms.order(values, out=order_t, flags=flags, check=False)
        if ev is not None:
            ev[1].record(stream)
        dms.discrete_gradient(order_t, lo, hi, out=rec, workspace=gws, mask=mask)
        if ev is not None:
            ev[2].record(stream)
        dms.critical_simplices(rec, dims, lo, hi, cap=cap, flags=flags, counts=counts_t, mask=mask)
        if ev is not None:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if int(flags.item()) != 0:
        raise RuntimeError("device flags set: %d" % int(flags.item()))
    stage = {"order": [], "gradient": [], "critical": []}
    for e in evs:
        stage["order"].append(e[0].elapsed_time(e[1]))
        stage["gradient"].append(e[1].elapsed_time(e[2]))
        stage["critical"].append(e[2].elapsed_time(e[3]))
    ms = {k: float(np.mean(v)) for k, v in stage.items()}
    # the equivalent gradient straight from the values (no order needed), same records
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dms.discrete_gradient_values(values, lo, hi, out=rec, workspace=gws, flags=flags, check=False)
    ev0.record(stream)
    for _ in range(3):
        dms.discrete_gradient_values(values, lo, hi, out=rec, workspace=gws, flags=flags, check=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_values_gradient = ev0.elapsed_time(ev1) / 3
    # the extraction without the mask (every record read), for comparison
    dms.critical_simplices(rec, dims, lo, hi, cap=cap, flags=flags, counts=counts_t)
    ev0.record(stream)
    for _ in range(3):
        dms.critical_simplices(rec, dims, lo, hi, cap=cap, flags=flags, counts=counts_t)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_critical_unmasked = ev0.elapsed_time(ev1) / 3
    # the extracted lists in filtration order (Section 2.1; the local sort
    # after extraction), all four dimensions; not part of the step
    sorted_lists = [torch.empty_like(lists[d]) for d in range(4)]
    for d in range(4):
        dms.critical_sort(lists[d], d, order_t, dims, out=sorted_lists[d], flags=flags, check=False)
    ev0.record(stream)
    for _ in range(3):
        for d in range(4):
            dms.critical_sort(lists[d], d, order_t, dims, out=sorted_lists[d], flags=flags, check=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_critical_sort = ev0.elapsed_time(ev1) / 3
    if int(flags.item()) != 0:
        raise RuntimeError("device flags set: %d" % int(flags.item()))
    ms_step = wall / args.steps * 1e3
    value = owned / (ms_step / 1e3) / 1e9

    # dominant call: dms_discrete_gradient (k_mark_zero + k_queue_reset + k_gradient +
    # k_gradient_queue on the same stream; the events bracket exactly these launches)
    stage_bytes = {k: ALG_BYTES[k] * owned for k in ALG_BYTES}
    # the masked extraction reads the mask and the flagged records only
    stage_bytes["critical"] = MASK_BYTES * owned + 16.0 * flagged
    dom = "gradient"
    achieved = stage_bytes[dom] / (ms[dom] / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic_gb(),
                "kernel": "dms_discrete_gradient: k_mark_zero + k_queue_reset + k_gradient<64,16> + k_gradient_queue",
                "kernel_ms": round(ms[dom], 3)}
    out = {
        "metric": "discrete-gradient Gvertices/s (order + gradient + critical) at 1024^3 owned f32",
        "value": round(value, 3),
        "unit": "Gvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "gauss1026_ghost: %dx%dx%d float32 block, owned %d^3 interior, "
                               "%d Gaussians + 1e-3 U[0,1) noise (seed 3)"
                               % (nx, ny, nz, args.owned, args.bumps),
                   "owned_vertices": owned, "critical_counts": [int(c) for c in cap]},
        "stage_ms": {k: round(v, 3) for k, v in ms.items()},
        "gradient_from_values_ms": round(ms_values_gradient, 3),
        "critical_unmasked_ms": round(ms_critical_unmasked, 3),
        "flagged_records": flagged,
        "critical_sort_ms": round(ms_critical_sort, 3),
        "stage_frac_hbm": {k: round(stage_bytes[k] / (ms[k] / 1e3) / 1e9 / HBM_PEAK_GBS, 4) for k in ms},
        "roofline": roofline,
        "input_gen_s": round(t_gen, 1),
    }
    del values, order_t, rec, lists
    torch.cuda.empty_cache()
    out["copy_gbs"] = copy_bandwidth(dev)
    if not args.no_extra:
        out["batched"] = bench_batched(dev, max(args.steps, 3))
        out["differentiable"] = bench_differentiable(dev, max(args.steps, 3))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(field, lo, hi, min(args.cpu_planes, args.owned))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
