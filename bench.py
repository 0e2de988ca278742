"""Throughput of the DD-CCLB step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-cpu] ...

Headline workload: the 3D droplet impacting a sphere, 256^3 periodic box
(sphere R = 60, droplet R = 40 moving at 0.02 towards it, density ratio 10,
90 deg walls), N = 2 phase sets on D3Q15 and a D3Q19 flow set, FP32 storage
and arithmetic: the largest single-GPU configuration of the paper's
setting. One "step" is one time step of the whole scheme (three kernel
launches: k_frac3d, k_mu3d, k_step3d). The JSON `value` is its node-MLUPS;
`roofline` prices the step against the 8 TB/s HBM peak with the algorithmic
bytes of one node update (populations read and written once, history read
and written once, psi and the wetting weight read once: 528 B at N = 2 in
FP32, 544 B counting the float64 rest planes the library keeps) over the
average step duration from HIP events on the library's stream.

Other legs in the same line: the 3D box in FP64 and with 16-bit population
storage, the 2D porous box (512 x 512, N = 3; it fits the 256 MB
memory-side cache, so its rate is not an HBM roofline figure) and the same
porous generator at 2048 x 2048 (streamed from HBM), the batch of 256
independent 2D boxes, and the adjoint sweep. Each leg carries its mass
drift, and its error against the FP64 oracle from this run (the 2048^2 box
is too large for the oracle here; its kernels are the ones the streaming
parity tests check).
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
KERNEL_SOURCES = {
    "2d": ["paper_2311_10314_amd/csrc/step2d.hip",
           "paper_2311_10314_amd/csrc/collide.hpp",
           "paper_2311_10314_amd/csrc/common.hpp",
           "paper_2311_10314_amd/csrc/lattice.hpp",
           "paper_2311_10314_amd/csrc/coef.hpp"],
    "3d": ["paper_2311_10314_amd/csrc/step3d.hip",
           "paper_2311_10314_amd/csrc/collide.hpp",
           "paper_2311_10314_amd/csrc/common.hpp",
           "paper_2311_10314_amd/csrc/lattice.hpp",
           "paper_2311_10314_amd/csrc/coef.hpp"],
}
# the 2D porous box at an HBM size (2048^2) runs the same sources
KERNEL_SOURCES["2dhbm"] = KERNEL_SOURCES["2d"]
HBM_2D_N = 2048
# element bytes (populations, fields) per precision
PREC_BYTES = {"fp64": (8, 8), "fp32": (4, 4), "fp16": (2, 4), "bf16": (2, 4)}
# The kernels of one step, as rocprofv3 names them (the 3D step is three
# launches: C_i from the pulled phase populations, the chemical potential,
# the node update; the 16-bit instances appear under their mangled names).
KERNEL_TAGS = {   # the 256^3 steps run in the streaming mode (3), 512^2 in 0
    ("3d", "fp32"): ["k_frac3d<2, ddcc::D3Q15, float, float, float, 3, 4>",
                     "k_mu3d<2, float, float, 4, true>",
                     "k_step3d<2, ddcc::D3Q15, ddcc::D3Q19, float, float, "
                     "float, 3, 4>"],
    ("3d", "fp64"): ["k_frac3d<2, ddcc::D3Q15, double, double, double, 3, 4>",
                     "k_mu3d<2, double, double, 4, true>",
                     "k_step3d<2, ddcc::D3Q15, ddcc::D3Q19, double, double, "
                     "double, 3, 4>"],
    ("3d", "fp16"): ["k_frac3dILi2ENS_5D3Q15EDF16_ffLi3ELi4E",
                     "k_mu3dILi2EDF16_fLi4ELb1E",
                     "k_step3dILi2ENS_5D3Q15ENS_5D3Q19EDF16_ffLi3ELi4E"],
    ("2d", "fp32"): ["k_step2d<3, float, float, float, 0, 8>"],
    ("2d", "fp64"): ["k_step2d<3, double, double, double, 0, 4>"],
    ("2dhbm", "fp32"): ["k_step2d<3, float, float, float, 3, 8>"],
    ("2dhbm", "fp64"): ["k_step2d<3, double, double, double, 3, 4>"],
}
HEAD_N = 256          # the 3D box of the headline
REDUCED_N = 48        # the same generator at 48^3 for the oracle legs


def algorithmic_bytes_per_node(N, dim, Qf, Qg, precision, rest64=False):
    """Bytes one node update must move: every population (N Qf + Qg) read
    and written once in the population storage type, the history (N d
    values phi C_i u, d(d+1)/2 of the symmetric flux tensor, P: in place)
    and the antisymmetric tensor T (d(d-1)/2, double-buffered) read and
    written once, psi and the N-1 wetting weights read once, in the field
    type. rest64: the N rest populations of the phase sets counted as the
    float64 the library keeps them in (so that storage rounding cannot
    change a phase's mass)."""
    pesz, fesz = PREC_BYTES[precision]
    pops = (N * Qf + Qg) * 2 * pesz
    if rest64:
        pops += N * 2 * (8 - pesz)
    hist = (N * dim + dim * (dim + 1) // 2 + 1) * 2
    tens = (dim * (dim - 1) // 2) * 2
    static = 1 + (N - 1)
    return pops + (hist + tens + static) * fesz


def _code_only(text):
    """C++ source without its comments and blank space, so that a change
    of comments alone does not mark the counters as stale."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(kind):
    """Hash of the code (comments and spacing removed) of the sources the
    step kernels of `kind` are built from."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kind, precision):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if
    they were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get("%s_%s" % (kind, precision))
    if not e or e.get("kernel_hash") != kernel_source_hash(kind):
        return None
    return e.get("bytes_per_launch")


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def rel_linf(a, b):
    import numpy as np
    scale = float(np.abs(b).max())
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def field_errors(got, ref, psi):
    """Relative L-inf of every C_i, of u and of P where psi >= 1e-2 (P =
    phi P / phi is round-off over a vanishing psi inside solids), and of
    phi P everywhere, against reference fields."""
    import numpy as np
    C, u, P = got
    Co, uo, Po = ref
    psi = np.asarray(psi)
    fl = psi >= 1e-2
    return {"rel_linf_C": max(rel_linf(C[i], Co[i]) for i in range(len(Co))),
            "rel_linf_u": rel_linf(u, uo),
            "rel_linf_P": rel_linf(P[fl], Po[fl]),
            "rel_linf_psiP": rel_linf(psi * P, psi * Po)}


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



COPY_RATE = True      # off in counter runs, whose 1 GiB calibration copy
                      # must be the largest copy of the run


def roofline(kind, precision, nodes, ms, N, dim, Qf, Qg, torch):
    """Roofline object of one step: algorithmic bytes of a step over its
    average duration (HIP events around the timed steps on the library's
    stream), the bytes with the float64 rest planes, the counter traffic (if
    taken on the current source) and the same-session copy rate of the same
    bytes."""
    bpn = algorithmic_bytes_per_node(N, dim, Qf, Qg, precision)
    bpn64 = algorithmic_bytes_per_node(N, dim, Qf, Qg, precision, True)
    per_launch = bpn * nodes
    achieved = per_launch / (ms * 1e-3) / 1e9
    copy = copy_rate(torch, bpn64 * nodes) if COPY_RATE else float("nan")
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(kind, precision),
            "kernels": KERNEL_TAGS.get((kind, precision)),
            "bytes_per_node": bpn,
            "algorithmic_bytes_per_launch": per_launch,
            "bytes_per_node_with_float64_rest": bpn64,
            "achieved_with_float64_rest": bpn64 * nodes / (ms * 1e-3) / 1e9,
            "copy_GBs": copy, "frac_of_copy": achieved / copy}


BATCH_ERR_STEPS = 20


def batch_check_instances(count):
    """Instances of the batch compared with the oracle: the three smallest
    and the largest."""
    from paper_2311_10314_amd import workloads as W
    wls = W.batched_instances(count)
    order = sorted(range(count), key=lambda i: wls[i].nodes)
    return [(i, wls[i]) for i in order[:3] + order[-1:]]


def oracle_leg(wl_small, steps, wl2d, steps2d, batch_count=0, threads=1):
    """The cpu_baseline leg: the FP64 oracle, untuned, on one pinned core,
    on a bounded sample of the headline workload (the same generator on a
    reduced box, the same work per node update), timed; its results are
    also the reference of the error columns (reduced 3D box after `steps`
    steps, 2D porous box after `steps2d` steps)."""
    import warnings

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    warnings.simplefilter("ignore")
    keep = os.sched_getaffinity(0)
    core = min(keep)
    try:
        os.sched_setaffinity(0, {core})
        with threadpool_limits(limits=threads):
            prm, geo, st = oracle.from_workload(wl_small)
            m0 = oracle.mass(st)
            t = time.perf_counter()
            st = oracle.run(prm, geo, st, steps)
            dt = time.perf_counter() - t
            ref3 = oracle.moments(prm, geo, st)
            drift3 = float(np.max(np.abs(oracle.mass(st) - m0) / np.abs(m0)))
            prm2, geo2, st2 = oracle.from_workload(wl2d)
            st2 = oracle.run(prm2, geo2, st2, steps2d)
            ref2 = oracle.moments(prm2, geo2, st2)
            refb = []
            if batch_count:
                for i, wb in batch_check_instances(batch_count):
                    pb, gb, sb = oracle.from_workload(wb)
                    sb = oracle.run(pb, gb, sb, BATCH_ERR_STEPS)
                    refb.append((i, wb, oracle.moments(pb, gb, sb)))
    finally:
        os.sched_setaffinity(0, keep)
    base = {"value": wl_small.nodes * steps / dt / 1e6, "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "sample": "%d steps of the %s box (%dx%dx%d, the headline's "
                      "generator with sizes scaled by %d/%d; same work per "
                      "node update), numpy float64, %d thread pinned to "
                      "core %d, %.1f s" % (
                          steps, wl_small.name, *wl_small.shape,
                          wl_small.shape[0], HEAD_N, threads, core, dt)}
    base.update(cpu_info())
    return base, {"sphere": ref3, "sphere_drift": drift3, "porous": ref2,
                  "batch": refb}


def sampled_full_size_error(wl, sim, count, hw=5, seed=256):
    """One more step of the full-size state against one oracle step on
    periodic windows around `count` sampled nodes (random, the wall layer,
    the droplet interface): a node's next state depends on the state
    within 4 nodes, so each window's centre is exact. Worst population
    error relative to the largest population at the centres."""
    import numpy as np

    import oracle
    from tests.helpers import unpack_state, window, window_state
    rng = np.random.default_rng(seed)
    shape = wl.shape
    pts = [tuple(int(rng.integers(0, n)) for n in shape)
           for _ in range(count // 2)]
    psi = np.asarray(wl.psi)
    C = np.asarray(wl.C0[0])
    for mask in ((psi > 0.2) & (psi < 0.8),
                 (C > 0.2) & (C < 0.8) & (psi > 0.9)):
        idx = np.argwhere(mask)
        pick = rng.choice(len(idx), size=min(count // 4, len(idx)),
                          replace=False)
        pts += [tuple(int(v) for v in idx[k]) for k in pick]
    s0 = unpack_state(sim, sim.save(), lazy=True)
    sim.step(1)
    s1 = unpack_state(sim, sim.save(), lazy=True)
    prm = oracle.Params(dim=wl.dim, lattice_f=wl.lattice_f,
                        lattice_g=wl.lattice_g, **wl.params)
    worst = 0.0
    c = (hw,) * len(shape)
    for center in pts:
        geo = oracle.Geometry(prm, window(psi, center, hw),
                              window(np.asarray(wl.cos_theta_iN), center,
                                     hw))
        st1 = oracle.step(prm, geo, window_state(wl, s0, center, hw))
        got = window_state(wl, s1, center, hw)
        for a, b in ((got.f, st1.f), (got.g, st1.g)):
            ref = b[(Ellipsis,) + c]
            worst = max(worst, float(np.abs(a[(Ellipsis,) + c] - ref).max()
                                     / np.abs(ref).max()))
    return {"rel_linf_populations": worst, "nodes": len(pts),
            "case": "one step after %d, windows of %d^%d" % (
                s0["t"], 2 * hw + 1, len(shape))}


def batch_errors(refs, count, torch):
    """The whole batch (FP32, graph step loop) for BATCH_ERR_STEPS steps,
    the checked instances against the oracle."""
    import numpy as np

    from paper_2311_10314_amd import workloads as W
    from paper_2311_10314_amd.ddcc import Batch
    b = Batch.from_workloads(W.batched_instances(count), "fp32")
    b.set_graph(10)
    m0 = {i: b.mass(i) for i, _, _ in refs}
    b.step(BATCH_ERR_STEPS)
    out = {}
    for i, wb, ref in refs:
        e = field_errors(b.read_moments(i), ref, wb.psi)
        e["mass_drift"] = float(np.max(np.abs(b.mass(i) - m0[i])
                                       / np.abs(m0[i])))
        e["shape"] = list(wb.shape)
        out["instance_%d" % i] = e
    b.close()
    out["steps"] = BATCH_ERR_STEPS
    return out


def gpu_errors(wl, precision, steps, ref, torch):
    """The library on a workload for `steps` steps against oracle fields,
    with its mass drift."""
    import numpy as np

    from paper_2311_10314_amd.ddcc import Sim
    sim = Sim.from_workload(wl, precision)
    m0 = sim.mass()
    sim.step(steps)
    got = sim.read_moments()
    drift = float(np.max(np.abs(sim.mass() - m0) / np.abs(m0)))
    sim.close()
    e = field_errors(got, ref, wl.psi)
    e.update({"mass_drift": drift, "steps": steps,
              "case": "%s %s" % (wl.name, "x".join(map(str, wl.shape)))})
    return e


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


def _counter_means(csv_path, counter, tags):
    """Sum over the kernels of `tags` (name substrings) of the mean counter
    value (KiB per dispatch), and the mean of the 1 GiB calibration copy
    (the largest buffer-copy dispatch) in one rocprofv3 counter run."""
    import csv
    with open(csv_path) as fh:
        rows = [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
    step, nd = 0.0, []
    for tag in tags:
        v = [float(r["Counter_Value"]) for r in rows
             if tag in r["Kernel_Name"]]
        if not v:
            raise SystemExit("%s: no %s dispatches of %s" % (csv_path,
                                                               counter, tag))
        step += sum(v) / len(v)
        nd.append(len(v))
    # the 1 GiB calibration copies: the largest copy dispatches of the run
    # (the runtime's copy kernel keeps one grid size for all large copies,
    # so they are told apart by their counter values)
    copies = [float(r["Counter_Value"]) for r in rows
              if "copyBuffer" in r["Kernel_Name"]]
    copy = []
    if copies:
        top = max(copies)
        copy = [v for v in copies if v >= 0.9 * top]
    if not copy or max(copy) < 1.0e5:
        raise SystemExit("%s: no %s dispatches of the 1 GiB copy (run with "
                         "--copy-calibration)" % (csv_path, counter))
    return step, sum(copy) / len(copy), nd


def traffic_summary(fetch_dir, write_dir, kind, precision):
    """Scale the FETCH_SIZE and WRITE_SIZE counters of a step kernel by what
    they read for a 1 GiB device copy in the same run, and record the HBM
    bytes per launch in profiles/hbm_traffic.json under the hash of the
    kernel sources (bench.py reports them only while the hash matches)."""
    from paper_2311_10314_amd import workloads as W
    if kind == "3d":
        wl = W.droplet_impact_sphere_3d(n=HEAD_N)
        geom = (2, 3, 15, 19)
    elif kind == "2dhbm":
        wl = W.porous_bands_2d(n=HBM_2D_N)
        geom = (3, 2, 9, 9)
    else:
        wl = W.porous_bands_2d(n=512)
        geom = (3, 2, 9, 9)
    tag = KERNEL_TAGS[(kind, precision)]
    f_step, f_copy, nd = _counter_means(
        os.path.join(fetch_dir, "run_counter_collection.csv"), "FETCH_SIZE",
        tag)
    w_step, w_copy, _ = _counter_means(
        os.path.join(write_dir, "run_counter_collection.csv"), "WRITE_SIZE",
        tag)
    gib_kib = 1024.0 * 1024.0
    ff, wf = gib_kib / f_copy, gib_kib / w_copy
    per_launch = (f_step * ff + w_step * wf) * 1024.0
    alg = algorithmic_bytes_per_node(*geom, precision) * wl.nodes
    entry = {"kernel": KERNEL_TAGS[(kind, precision)],
             "workload": "%s %s" % (wl.name, "x".join(map(str, wl.shape))),
             "kernel_hash": kernel_source_hash(kind),
             "dispatches": nd,
             "fetch_kib_per_dispatch": f_step,
             "write_kib_per_dispatch": w_step,
             "copy_fetch_kib_for_1GiB": f_copy,
             "copy_write_kib_for_1GiB": w_copy,
             "fetch_factor": ff, "write_factor": wf,
             "read_bytes_per_launch": f_step * ff * 1024.0,
             "write_bytes_per_launch": w_step * wf * 1024.0,
             "bytes_per_launch": per_launch,
             "algorithmic_bytes_per_launch": alg,
             "ratio_to_algorithmic": per_launch / alg}
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    t["%s_%s" % (kind, precision)] = entry
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(entry, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps of the headline (256^3 FP32)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=HEAD_N,
                    help="edge of the headline's 3D box")
    ap.add_argument("--leg-steps", type=int, default=50,
                    help="timed steps of the other 3D precisions")
    ap.add_argument("--porous-steps", type=int, default=2000)
    ap.add_argument("--cpu-steps", type=int, default=160,
                    help="oracle steps on the reduced 3D box (also the "
                         "steps of the error columns there)")
    ap.add_argument("--samples", type=int, default=12,
                    help="sampled nodes of the full-size one-step check")
    ap.add_argument("--skip-cpu", action="store_true",
                    help="no oracle (no cpu_baseline, no error columns)")
    ap.add_argument("--batch", type=int, default=256,
                    help="also time this many batched instances (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--adjoint", type=int, default=256,
                    help="also time the adjoint sweep on the n x n channel "
                         "(0: skip)")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--precisions", default="fp32,fp64,fp16,bf16",
                    help="3D precisions to time (the first is not repeated)")
    ap.add_argument("--no-2d", action="store_true")
    ap.add_argument("--porous-hbm", type=int, default=HBM_2D_N,
                    help="side of the 2D porous box timed at an HBM size "
                         "(0: skip)")
    ap.add_argument("--porous-hbm-steps", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--sweep", metavar="OUT_JSON", nargs="?", const="",
                    default=None,
                    help="run only the 2D roofline sweep over grid sizes, "
                         "phase counts and precisions")
    ap.add_argument("--traffic-summary", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "KIND", "PRECISION"),
                    help="write profiles/hbm_traffic.json from two "
                         "rocprofv3 counter runs (no GPU needed); KIND is "
                         "3d, 2d or 2dhbm")
    a = ap.parse_args()
    if a.traffic_summary:
        traffic_summary(*a.traffic_summary)
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
    from paper_2311_10314_amd import workloads as W
    if a.copy_calibration:
        global COPY_RATE
        COPY_RATE = False
        copy_calibration(torch)

    # ---- headline: 3D box, FP32 ------------------------------------------
    wl = W.droplet_impact_sphere_3d(n=a.n)
    precs = [p for p in a.precisions.split(",") if p]
    head_prec = precs[0]
    print("headline: %s %s, %d warmup + %d steps" % (
        wl.name, "x".join(map(str, wl.shape)), a.warmup, a.steps),
        file=sys.stderr, flush=True)
    sim, ms, drift = time_gpu(wl, head_prec, a.steps, a.warmup, torch)
    sampled = None
    if not a.skip_cpu and a.samples > 0:
        sampled = sampled_full_size_error(wl, sim, a.samples)
        print("  full-size sampled one-step check: %s" % sampled,
              file=sys.stderr, flush=True)
    sim.close()
    head_roof = roofline("3d", head_prec, wl.nodes, ms, 2, 3, 15, 19, torch)
    print("  %s: %.4f ms/step, %.0f MLUPS, %.0f GB/s algorithmic "
          "(%.3f of peak)" % (head_prec, ms, wl.nodes / (ms * 1e-3) / 1e6,
                              head_roof["achieved"], head_roof["frac"]),
          file=sys.stderr, flush=True)
    legs3 = {}
    for prec in precs[1:]:
        s2, ms2, dr2 = time_gpu(wl, prec, a.leg_steps, a.warmup, torch)
        s2.close()
        legs3[prec] = {"value": wl.nodes / (ms2 * 1e-3) / 1e6,
                       "unit": "MLUPS", "ms_per_step": ms2,
                       "steps": a.leg_steps, "mass_drift": dr2,
                       "roofline": roofline("3d", prec, wl.nodes, ms2, 2, 3,
                                            15, 19, torch)}
        print("  %s: %.4f ms/step" % (prec, ms2), file=sys.stderr,
              flush=True)

    # ---- 2D porous box (cache-resident) ------------------------------------
    wl2 = W.porous_bands_2d(n=512)
    porous = None
    if not a.no_2d:
        porous = {"workload": "porous_bands_2d 512x512, N=3 (+1 flow set), "
                              "D2Q9, 40 disks, rho 1:10:100",
                  "cache_resident": True,
                  "note": "about 110 MB (FP32) / 205 MB (FP64) per step fit "
                          "the 256 MB memory-side cache: not an HBM "
                          "roofline measurement"}
        for prec in ("fp32", "fp64"):
            s2, ms2, dr2 = time_gpu(wl2, prec, a.porous_steps, 50, torch)
            s2.close()
            r = roofline("2d", prec, wl2.nodes, ms2, 3, 2, 9, 9, torch)
            r["bound"] = "cache"
            porous[prec] = {"value": wl2.nodes / (ms2 * 1e-3) / 1e6,
                            "set_mlups": 4 * wl2.nodes / (ms2 * 1e-3) / 1e6,
                            "unit": "MLUPS", "ms_per_step": ms2,
                            "steps": a.porous_steps, "mass_drift": dr2,
                            "roofline": r}
            print("  porous 512^2 %s: %.4f ms/step" % (prec, ms2),
                  file=sys.stderr, flush=True)

    # ---- 2D porous box at an HBM size (streaming step mode) ----------------
    porous_hbm = None
    if not a.no_2d and a.porous_hbm > 0:
        n3 = a.porous_hbm
        wl3 = W.porous_bands_2d(n=n3)
        porous_hbm = {"workload": "porous_bands_2d %dx%d, N=3 (+1 flow set), "
                                  "D2Q9, rho 1:10:100" % (n3, n3),
                      "note": "streams from HBM (the library's streaming "
                              "step mode); the same kernels as the 1024^2 "
                              "and 790x830 streaming parity tests; traffic "
                              "from the counter run of the 2048^2 box"}
        for prec in ("fp32", "fp64"):
            s3, ms3, dr3 = time_gpu(wl3, prec, a.porous_hbm_steps, 10, torch)
            s3.close()
            r = roofline("2dhbm", prec, wl3.nodes, ms3, 3, 2, 9, 9, torch)
            if n3 != HBM_2D_N:  # counters were taken on the 2048^2 box
                r["traffic"] = None
            porous_hbm[prec] = {"value": wl3.nodes / (ms3 * 1e-3) / 1e6,
                                "unit": "MLUPS", "ms_per_step": ms3,
                                "steps": a.porous_hbm_steps,
                                "mass_drift": dr3, "roofline": r}
            print("  porous %d^2 %s: %.4f ms/step, %.0f GB/s algorithmic "
                  "(%.3f of peak)" % (n3, prec, ms3, r["achieved"], r["frac"]),
                  file=sys.stderr, flush=True)
        del wl3

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

    # ---- cpu_baseline leg: the oracle, and the error columns ---------------
    cpu = None
    err = None
    if not a.skip_cpu:
        small = W.droplet_impact_sphere_3d(n=REDUCED_N)
        print("cpu baseline: oracle on %s %s, %d steps, one core" % (
            small.name, "x".join(map(str, small.shape)), a.cpu_steps),
            file=sys.stderr, flush=True)
        cpu, ref = oracle_leg(small, a.cpu_steps, wl2, 10,
                              a.batch if batched else 0)
        for prec in precs:
            e = gpu_errors(small, prec, a.cpu_steps, ref["sphere"], torch)
            e["oracle_mass_drift"] = ref["sphere_drift"]
            if prec == head_prec:
                err = {"reduced_box": e, "full_size_sampled": sampled}
            else:
                legs3[prec]["error_vs_oracle"] = e
            print("  %s error on the reduced box: %s" % (prec, e),
                  file=sys.stderr, flush=True)
        if porous:
            for prec in ("fp32", "fp64"):
                porous[prec]["error_vs_oracle"] = gpu_errors(
                    wl2, prec, 10, ref["porous"], torch)
        if batched:
            batched["error_vs_oracle"] = batch_errors(ref["batch"],
                                                      a.batch, torch)
    line = {
        "metric": METRIC,
        "value": wl.nodes / (ms * 1e-3) / 1e6, "unit": "MLUPS",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "fp64": "f64",
                                       "fp16": "f32", "bf16": "f32"}[head_prec],
        "data": "synthetic",
        "config": {"workload": "droplet_impact_sphere_3d: %d^3 periodic, "
                               "N=2 phase sets (D3Q15) + flow set (D3Q19), "
                               "sphere R=%g, droplet R=%g at 0.02, rho "
                               "10:1, %s storage" % (
                                   a.n, 60 * a.n / 256, 40 * a.n / 256,
                                   head_prec),
                   "nodes": wl.nodes, "phases": 2, "precision": head_prec},
        "set_mlups": 3 * wl.nodes / (ms * 1e-3) / 1e6,
        "mass_drift": drift,
        "roofline": head_roof,
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "sphere3d": legs3,
        "porous2d": porous,
        "porous2d_hbm": porous_hbm,
        "batched": batched,
        "adjoint": adjoint,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
