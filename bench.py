"""Throughput of the fused DD-CCLB step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512] [--skip-cpu]

Workload: the 2D porous medium of the paper's setting (512 x 512 periodic
box, 40 seeded disks with radii U[10, 30], three vertical phase bands,
per-obstacle contact angles U[45, 135] deg, densities 1:10:100, body force
density 1e-6), N = 3 phase sets + 1 flow set on D2Q9. One "step" is one
time step of the whole scheme (one fused kernel launch). Both FP32 and FP64
are timed; the JSON `value` is the FP32 figure and `fp64` holds the other.
The 3D leg (`sphere3d`: a droplet impacting a sphere, D3Q15 phase sets and a
D3Q19 flow set, N = 2, n^3 box) is timed in FP32, FP64 and the two 16-bit
population storages, each with its error against the FP64 oracle on the
same case at 32^3.

MLUPS counts lattice-node updates per second, each update covering all N + 1
distribution sets. `roofline.achieved` is the algorithmic HBM bytes of one
node update (populations read + written once, history read + written once,
static fields read once) times the nodes of one launch, divided by the
average launch duration measured with HIP events on the library's stream.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS (all distribution sets) and % of HBM roofline, "
          "FP32 vs FP64 at stated error")
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
KERNEL_SOURCES = ["paper_2311_10314_amd/csrc/step2d.hip",
                  "paper_2311_10314_amd/csrc/collide.hpp",
                  "paper_2311_10314_amd/csrc/common.hpp",
                  "paper_2311_10314_amd/csrc/lattice.hpp",
                  "paper_2311_10314_amd/csrc/coef.hpp"]


PREC_BYTES = {"fp64": (8, 8), "fp32": (4, 4), "fp16": (2, 4), "bf16": (2, 4)}


def algorithmic_bytes_per_node(N, dim, Qf, Qg, precision):
    """Populations (N Qf + Qg) read and written once (the N rest populations
    of the phase sets are float64 in every precision, the moving ones and the
    flow set in the population storage type), history
    (N d + d(d+1)/2 + 1 in place, d(d-1)/2 double-buffered) read and written
    once, psi and N-1 wetting cosines read once (field storage type)."""
    pesz, fesz = PREC_BYTES[precision]
    pops = (N * (Qf - 1) + Qg) * 2 * pesz + N * 2 * 8
    hist = (N * dim + dim * (dim + 1) // 2 + 1) * 2
    tens = (dim * (dim - 1) // 2) * 2
    static = 1 + (N - 1)
    return pops + (hist + tens + static) * fesz


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if
    they were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(precision)
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def make_workload(n):
    from paper_2311_10314_amd import workloads as W
    return W.porous_bands_2d(n=n)


def sphere_leg(n, steps, warmup, torch, precisions):
    """3D leg: the sphere / impacting-droplet box (D3Q15 phase sets, D3Q19
    flow set, N = 2) at n^3, with each precision's error against the FP64
    oracle after 40 steps of the same case at 32^3."""
    import numpy as np

    from paper_2311_10314_amd import workloads as W
    from paper_2311_10314_amd.ddcc import Sim
    wl = W.droplet_impact_sphere_3d(n=n)
    small = W.droplet_impact_sphere_3d(n=32)
    ref = None
    out = {}
    for prec in precisions:
        sim, ms, drift = time_gpu(wl, prec, steps, warmup, torch)
        sim.close()
        bpn = algorithmic_bytes_per_node(2, 3, 15, 19, prec)
        achieved = bpn * wl.nodes / (ms * 1e-3) / 1e9
        if ref is None:
            import oracle
            prm, geo, st = oracle.from_workload(small)
            st = oracle.run(prm, geo, st, 40)
            ref = oracle.moments(prm, geo, st)
        s2 = Sim.from_workload(small, prec)
        s2.step(40)
        C, u, _ = s2.read_moments()
        s2.close()
        Co, uo, _ = ref
        err = {"rel_linf_C": max(float(np.abs(C[i] - Co[i]).max() /
                                       np.abs(Co[i]).max())
                                 for i in range(len(Co))),
               "rel_linf_u": float(np.abs(u - uo).max() / np.abs(uo).max()),
               "case": "32^3, 40 steps"}
        out[prec] = {"value": wl.nodes / (ms * 1e-3) / 1e6,
                     "unit": "MLUPS", "ms_per_step": ms, "mass_drift": drift,
                     "bytes_per_node": bpn, "achieved_GBs": achieved,
                     "frac": achieved / HBM_PEAK_GBS, "steps": steps,
                     "error_vs_oracle": err}
        print("  sphere3d %d^3 %s: %.4f ms/step, %.0f MLUPS, %.0f GB/s%s" % (
            n, prec, ms, out[prec]["value"], achieved,
            ", C %.1e u %.1e" % (err["rel_linf_C"], err["rel_linf_u"])),
            file=sys.stderr, flush=True)
    return out


def batched_leg(count, steps, torch, graph_steps=50):
    """Batched leg: `count` independent 2D N = 2 instances of uneven sizes
    (sides from {64, 96, 128, 192, 256}, seeded disks and droplets) advanced
    by one persistent launch per step, the tile height picked by the
    library's autotuner and the steps replayed from HIP graphs of
    `graph_steps` steps. FP32."""
    import numpy as np

    from paper_2311_10314_amd import workloads as W
    from paper_2311_10314_amd.ddcc import Batch
    wls = W.batched_instances(count)
    stream = torch.cuda.Stream()
    b = Batch.from_workloads(wls, "fp32", stream=stream.cuda_stream)
    ty = b.autotune(5)
    b.set_graph(graph_steps)
    m0 = [b.mass(i) for i in range(count)]
    b.step(2 * graph_steps)
    b.sync()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    b.step(steps)
    t1.record(stream)
    t1.synchronize()
    ms = t0.elapsed_time(t1) / steps
    drift = max(float((np.abs(b.mass(i) - m0[i]) / np.abs(m0[i])).max())
                for i in range(count))
    nodes = b.nodes
    b.close()
    bpn = algorithmic_bytes_per_node(2, 2, 9, 9, "fp32")
    achieved = bpn * nodes / (ms * 1e-3) / 1e9
    out = {"value": nodes / (ms * 1e-3) / 1e6, "unit": "MLUPS",
           "instances": count, "nodes": nodes, "ms_per_step": ms,
           "steps": steps, "tile_rows": ty, "graph_steps": graph_steps,
           "mass_drift": drift, "bytes_per_node": bpn,
           "achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS}
    print("  batched %d instances (%d nodes): %.4f ms/step, %.0f MLUPS, "
          "%.0f GB/s, tile rows %d" % (count, nodes, ms, out["value"],
                                       achieved, ty), file=sys.stderr,
          flush=True)
    return out


def adjoint_leg(n, steps, interval, torch):
    """Adjoint sweep on the wavy channel (256 x 256, N = 2, per-node angle
    field): wall time of ddcc_adjoint (forward sweep with checkpoints,
    segment recomputation and the reverse sweep) against the forward steps
    alone, in FP32 and FP64, with the FP32 gradient's deviation from the
    FP64 one and the FP64 gradient against central differences along a
    smooth random direction of the angle field."""
    import numpy as np

    from paper_2311_10314_amd import workloads as W
    from paper_2311_10314_amd.ddcc import Sim
    wl = W.adjoint_channel_2d(n=n, steps=steps)
    out = {"workload": "adjoint_channel_2d %dx%d N=2, %d steps, checkpoints "
                       "every %d" % (n, n, steps, interval)}
    grads = {}
    for prec in ("fp32", "fp64"):
        sim = Sim.from_workload(wl, prec)
        state = sim.save()
        sim.step(10)
        sim.load(state)
        sim.sync()
        t = time.perf_counter()
        sim.step(steps)
        sim.sync()
        fwd = time.perf_counter() - t
        sim.load(state)
        t = time.perf_counter()
        J, gc, gp = sim.adjoint(steps, interval)
        adj = time.perf_counter() - t
        grads[prec] = (J, gc, gp, sim, state)
        out[prec] = {"J": J, "seconds": adj,
                     "ms_per_step": adj / steps * 1e3,
                     "forward_ms_per_step": fwd / steps * 1e3}
        print("  adjoint %s: %.3f s for %d steps (%.3f ms/step; forward "
              "alone %.3f ms/step), J = %.10f" % (prec, adj, steps,
                                                  adj / steps * 1e3,
                                                  fwd / steps * 1e3, J),
              file=sys.stderr, flush=True)
    J, gc, gp, sim, state = grads["fp64"]
    gc32, gp32 = grads["fp32"][1], grads["fp32"][2]
    out["fp32_vs_fp64"] = {
        "rel_linf_grad_cos": float(np.abs(gc32 - gc).max() / np.abs(gc).max()),
        "rel_linf_grad_psi": float(np.abs(gp32 - gp).max() / np.abs(gp).max())}
    psi0 = np.asarray(wl.psi)
    cos0 = np.asarray(wl.cos_theta_iN).reshape(gc.shape)
    v = W.smooth_angle_field(wl.shape, 7, lo=-1.0, hi=1.0)[None]

    def value(h):
        sim.init_geometry(psi0, cos0 + h * v)
        sim.load(state)
        sim.step(steps)
        return sim.objective()

    h = 2e-3
    d1 = (value(h) - value(-h)) / (2 * h)
    d2 = (value(h / 2) - value(-h / 2)) / h
    fd = (4.0 * d2 - d1) / 3.0
    ad = float((gc * v).sum())
    out["fd_check_fp64"] = {"adjoint": ad, "finite_differences": fd,
                            "rel_err": abs(fd - ad) / abs(ad)}
    for p in grads.values():
        p[3].close()
    return out


def copy_calibration(torch, mib=1024):
    """A plain device copy of known size, for scaling the HBM byte counters
    (FETCH_SIZE / WRITE_SIZE) read on the step kernel."""
    a = torch.empty(mib * 1024 * 1024 // 4, dtype=torch.float32,
                    device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copy calibration: 3 copies of %d MiB" % mib, file=sys.stderr,
          flush=True)


def copy_rate(torch, nbytes, reps=None):
    """Streaming reference measured in the same session: GB/s of the
    runtime's device-to-device copy moving `nbytes` per copy (nbytes / 2
    read, nbytes / 2 written), alternating between two buffers so that
    nothing is re-read from a warm cache that a step would not also have."""
    half = max(1, int(nbytes) // 2 // 4)
    a = torch.empty(half, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.zero_()
    b.zero_()
    if reps is None:
        reps = max(10, min(400, int(20e9 // max(nbytes, 1))))
    for i in range(4):
        (b if i % 2 == 0 else a).copy_(a if i % 2 == 0 else b)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for i in range(reps):
        (b if i % 2 == 0 else a).copy_(a if i % 2 == 0 else b)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * half * 4 / (ms * 1e-3) / 1e9


def sweep(torch, out_path=None):
    """Roofline sweep of the 2D step over grid sizes, phase counts and
    precisions: porous_bands_2d (N = 3) at 512^2 to 4096^2 and
    disk_on_droplet_2d (N = 2) at 512^2 to 8192^2, FP32 and FP64. Each point:
    ms per step (HIP events over enough steps to move about 20 GB),
    node-MLUPS, algorithmic GB/s and its fraction of the 8 TB/s peak, and the
    same-session copy rate for the same number of bytes."""
    from paper_2311_10314_amd import workloads as W
    points = [("porous_bands_2d", n) for n in (512, 2048, 4096)] + \
             [("disk_on_droplet_2d", n) for n in (512, 2048, 4096, 8192)]
    rows = []
    for name, n in points:
        t = time.perf_counter()
        wl = getattr(W, name)(n=n)
        print("sweep: %s %d^2 N=%d generated in %.1f s" % (
            name, n, wl.nphase, time.perf_counter() - t), file=sys.stderr,
            flush=True)
        for prec in ("fp32", "fp64"):
            bpn = algorithmic_bytes_per_node(wl.nphase, 2, 9, 9, prec)
            per = bpn * wl.nodes
            steps = max(10, min(20000, int(20e9 // per)))
            sim, ms, drift = time_gpu(wl, prec, steps, 5, torch)
            sim.close()
            gbs = per / (ms * 1e-3) / 1e9
            cp = copy_rate(torch, per)
            r = {"workload": name, "n": n, "phases": wl.nphase,
                 "precision": prec, "steps": steps, "ms_per_step": ms,
                 "mlups": wl.nodes / (ms * 1e-3) / 1e6,
                 "bytes_per_node": bpn, "algorithmic_GBs": gbs,
                 "frac_of_peak": gbs / HBM_PEAK_GBS, "copy_GBs": cp,
                 "frac_of_copy": gbs / cp, "mass_drift": drift}
            rows.append(r)
            print("  %-18s %5d^2 N=%d %s: %8.4f ms/step %7.0f MLUPS %6.0f "
                  "GB/s (%.0f %% of peak; copy of the same bytes %.0f GB/s, "
                  "%.0f %%)" % (name, n, wl.nphase, prec, ms, r["mlups"], gbs,
                                100 * r["frac_of_peak"], cp,
                                100 * r["frac_of_copy"]), file=sys.stderr,
                  flush=True)
        del wl
    if out_path:
        with open(out_path, "w") as fh:
            json.dump(rows, fh, indent=1)
            fh.write("\n")
    print(json.dumps({"sweep": rows}))
    return rows


STEP_KERNEL = {"fp32": "float, float, float", "fp64": "double, double, double"}


def _counter_means(csv_path, counter, precision, nphase):
    """Mean counter value (KiB per dispatch) of the step kernel and of the
    1 GiB calibration copy (the largest buffer-copy dispatch) in one
    rocprofv3 counter run."""
    import csv
    step, copy = [], []
    tag = "k_step2d<%d, %s, 0, " % (nphase, STEP_KERNEL[precision])
    with open(csv_path) as fh:
        rows = [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
    for r in rows:
        if tag in r["Kernel_Name"]:
            step.append(float(r["Counter_Value"]))
    # the 1 GiB calibration copies: the largest copy dispatches of the run
    # (the runtime's copy kernel keeps one grid size for all large copies,
    # so they are told apart by their counter values)
    copies = [float(r["Counter_Value"]) for r in rows
              if "copyBuffer" in r["Kernel_Name"]]
    if copies:
        top = max(copies)
        copy = [v for v in copies if v >= 0.9 * top]
    if not step or not copy or max(copy) < 1.0e5:
        raise SystemExit("%s: no %s dispatches of the step kernel or of the "
                         "1 GiB copy (run with --copy-calibration)"
                         % (csv_path, counter))
    return sum(step) / len(step), sum(copy) / len(copy), len(step)


def traffic_summary(fetch_dir, write_dir, precision, n):
    """Scale the FETCH_SIZE and WRITE_SIZE counters of the step kernel by
    what they read for a 1 GiB device copy in the same run, and record the
    HBM bytes per launch in profiles/hbm_traffic.json under the hash of the
    kernel sources (bench.py reports them only while the hash matches)."""
    wl = make_workload(n)
    N = wl.nphase
    f_step, f_copy, nd = _counter_means(
        os.path.join(fetch_dir, "run_counter_collection.csv"), "FETCH_SIZE",
        precision, N)
    w_step, w_copy, _ = _counter_means(
        os.path.join(write_dir, "run_counter_collection.csv"), "WRITE_SIZE",
        precision, N)
    gib_kib = 1024.0 * 1024.0
    ff, wf = gib_kib / f_copy, gib_kib / w_copy
    per_launch = (f_step * ff + w_step * wf) * 1024.0
    ty = 4 if precision == "fp64" else 8   # the library's default tiles
    entry = {"kernel": "k_step2d<%d, %s, 0, %d>" % (N, STEP_KERNEL[precision],
                                                     ty),
             "workload": "porous_bands_2d %dx%d N=%d" % (n, n, N),
             "kernel_hash": kernel_source_hash(),
             "dispatches": nd,
             "fetch_kib_per_dispatch": f_step,
             "write_kib_per_dispatch": w_step,
             "copy_fetch_kib_for_1GiB": f_copy,
             "copy_write_kib_for_1GiB": w_copy,
             "fetch_factor": ff, "write_factor": wf,
             "read_bytes_per_launch": f_step * ff * 1024.0,
             "write_bytes_per_launch": w_step * wf * 1024.0,
             "bytes_per_launch": per_launch,
             "algorithmic_bytes_per_launch":
                 algorithmic_bytes_per_node(N, 2, 9, 9, precision) * wl.nodes}
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    t[precision] = entry
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
        fh.write("\n")
    print(json.dumps(entry, indent=1))


def time_gpu(wl, precision, steps, warmup, torch, tile=0):
    from paper_2311_10314_amd.ddcc import Sim
    stream = torch.cuda.Stream()
    sim = Sim.from_workload(wl, precision, stream=stream.cuda_stream)
    if tile:
        sim.set_tile(0, tile)
    m0 = sim.mass()
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    sim.step(steps)
    t1.record(stream)
    t1.synchronize()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    try:
        m1 = sim.mass()
        drift = float(max(abs(a - b) / abs(b) for a, b in zip(m1, m0)))
    except Exception as e:  # a non-finite state is reported, not hidden
        print("mass check failed: %s" % e, file=sys.stderr, flush=True)
        drift = None
    return sim, ms / steps, drift


def error_vs_oracle(wl, steps):
    """Relative L-inf of C_i and u after `steps` steps, GPU vs oracle."""
    import numpy as np

    import oracle
    from paper_2311_10314_amd.ddcc import Sim
    prm, geo, st = oracle.from_workload(wl)
    st = oracle.run(prm, geo, st, steps)
    Co, uo, _ = oracle.moments(prm, geo, st)
    out = {}
    for prec in ("fp64", "fp32"):
        sim = Sim.from_workload(wl, prec)
        sim.step(steps)
        C, u, _ = sim.read_moments()
        eC = max(float(np.abs(C[i] - Co[i]).max() / np.abs(Co[i]).max())
                 for i in range(len(Co)))
        eu = float(np.abs(u - uo).max() / np.abs(uo).max())
        out[prec] = {"rel_linf_C": eC, "rel_linf_u": eu, "steps": steps}
        sim.close()
    return out


def cpu_baseline(wl, steps):
    """The FP64 oracle, untuned, on a bounded sample of the same workload:
    `steps` time steps of the full 512 x 512 box, one thread."""
    import warnings

    from threadpoolctl import threadpool_limits

    import oracle
    warnings.simplefilter("ignore")
    with threadpool_limits(limits=1):
        prm, geo, st = oracle.from_workload(wl)
        t = time.perf_counter()
        oracle.run(prm, geo, st, steps)
        dt = time.perf_counter() - t
    return {"value": wl.nodes * steps / dt / 1e6, "unit": "MLUPS",
            "cores": 1, "kind": "oracle",
            "sample": "%d steps of the full %dx%d N=%d box, numpy float64, "
                      "1 thread, %.1f s" % (steps, wl.shape[1], wl.shape[0],
                                             wl.nphase, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--cpu-steps", type=int, default=64)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--sphere", type=int, default=256,
                    help="also time the 3D sphere box at this n (0: skip)")
    ap.add_argument("--sphere-steps", type=int, default=100)
    ap.add_argument("--batch", type=int, default=256,
                    help="also time this many batched instances (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--adjoint", type=int, default=256,
                    help="also time the adjoint sweep on the n x n channel "
                         "(0: skip)")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--sweep", metavar="OUT_JSON", nargs="?", const="",
                    default=None,
                    help="run only the 2D roofline sweep over grid sizes, "
                         "phase counts and precisions")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR",
                                                           "WRITE_DIR"),
                    help="write profiles/hbm_traffic.json from two "
                         "rocprofv3 counter runs (no GPU needed)")
    ap.add_argument("--precision", default="both",
                    choices=["both", "fp32", "fp64"])
    a = ap.parse_args()
    if a.traffic_summary:
        traffic_summary(a.traffic_summary[0], a.traffic_summary[1],
                        "fp64" if a.precision == "fp64" else "fp32", a.n)
        return 0
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU "
              "path (a grid would be cut into slabs along its slowest axis, "
              "one per GPU, exchanging the crossing populations and a "
              "2-cell C halo every step)", file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    if a.sweep is not None:
        sweep(torch, a.sweep or None)
        return 0
    wl = make_workload(a.n)
    N = wl.nphase
    res = {}
    if a.copy_calibration:
        copy_calibration(torch)
    precs = (("fp32", 4), ("fp64", 8))
    if a.precision != "both":
        precs = tuple(x for x in precs if x[0] == a.precision)
    for prec, esz in precs:
        print("timing %s: %d warmup + %d steps on %s" % (prec, a.warmup,
                                                         a.steps, wl.shape),
              file=sys.stderr, flush=True)
        sim, ms, drift = time_gpu(wl, prec, a.steps, a.warmup, torch,
                                  a.tile)
        sim.close()
        bpn = algorithmic_bytes_per_node(N, 2, 9, 9, prec)
        per_launch = bpn * wl.nodes
        achieved = per_launch / (ms * 1e-3) / 1e9
        traffic = measured_traffic(prec)
        copy = copy_rate(torch, per_launch)
        res[prec] = {
            "value": wl.nodes / (ms * 1e-3) / 1e6,
            "set_mlups": (N + 1) * wl.nodes / (ms * 1e-3) / 1e6,
            "ms_per_step": ms,
            "mass_drift": drift,
            "roofline": {"bound": "hbm", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": traffic,
                         "copy_GBs": copy,
                         "frac_of_copy": achieved / copy,
                         "algorithmic_bytes_per_launch": per_launch,
                         "bytes_per_node": bpn},
        }
        print("  %s: %.4f ms/step, %.0f MLUPS, %.0f GB/s (copy of the same "
              "bytes: %.0f GB/s)" % (prec, ms, res[prec]["value"], achieved,
                                    copy), file=sys.stderr, flush=True)
    sphere = None
    if a.sphere:
        print("timing the 3D sphere box at %d^3" % a.sphere, file=sys.stderr,
              flush=True)
        sphere = sphere_leg(a.sphere, a.sphere_steps, 10, torch,
                            tuple(p for p, _ in precs) + ("fp16", "bf16"))
    batched = None
    if a.batch:
        print("timing %d batched instances" % a.batch, file=sys.stderr,
              flush=True)
        batched = batched_leg(a.batch, a.batch_steps, torch)
    adjoint = None
    if a.adjoint:
        print("timing the adjoint sweep on the %d^2 channel" % a.adjoint,
              file=sys.stderr, flush=True)
        adjoint = adjoint_leg(a.adjoint, a.adjoint_steps, 100, torch)
    err = None
    cpu = None
    if not a.skip_cpu:
        print("error vs oracle (10 steps) and cpu baseline", file=sys.stderr,
              flush=True)
        err = error_vs_oracle(wl, 10)
        cpu = cpu_baseline(wl, a.cpu_steps)
    if "fp32" not in res:
        print(json.dumps({"fp64": res["fp64"], "sphere3d": sphere,
                          "batched": batched, "adjoint": adjoint}))
        return 0
    f32 = res["fp32"]
    line = {
        "metric": METRIC, "value": f32["value"], "unit": "MLUPS",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": f32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "porous_bands_2d: %dx%d periodic, N=3 "
                               "(+1 flow set), D2Q9, 40 disks, rho 1:10:100"
                               % (a.n, a.n),
                   "nodes": wl.nodes, "phases": N, "precision": "fp32"},
        "set_mlups": f32["set_mlups"],
        "mass_drift": f32["mass_drift"],
        "roofline": f32["roofline"],
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "fp64": res.get("fp64"),
        "sphere3d": sphere,
        "batched": batched,
        "adjoint": adjoint,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
