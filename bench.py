"""Benchmark of the CFNEB band step on one MI355X.

Workload: graphite to cubic-diamond-like Tersoff carbon band, 98,304 atoms per
image, 24 initial images (adaptive insertion up to 40, checked every 20 steps),
15 GPa hydrostatic pressure through the rotation-free cell filter, FP32 pair and
three-body arithmetic with FP64 sums, band, cell filter and FIRE in FP64.

A step is one pass of the whole band step (every moving image: geometry, cell
list, neighbour list, forces, virial, cell filter; then tangents, springs,
climbing image, FIRE, and the adaptive-image check).  value = atoms x moving
images x steps / seconds over exactly --steps steps, inputs resident in HBM.

Prints one JSON line.  Extra objects: "roofline" for the kernel that takes the
most device time (from a second, profiled pass of the same workload with HIP
events around every phase on the band's stream, less the time two events take
around a phase that launches nothing) and "cpu_baseline" (the FP64
oracle on the host cores, on a bounded sample of the same workload).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.
# The kernels are built with packed FP32 disabled, so the unpacked rate is the ceiling.
VALU_FP32_PEAK_TFLOPS = 78.6

# Algorithmic work per unit of each phase (bytes that must cross HBM at least once).
#   rows = (atoms + 3) per moving image; atoms = atoms per moving image
#   Tersoff flops: 60 per directed bond + 80 per bond pair (triplet) for energy and forces
ALGO = {
    # per row: read X of the image and its two neighbours 72 B + F 12 B + v 24 B
    "dots": dict(bound="hbm", per="row", bytes=108),
    # per atom: read R~ 24 B and R_ref 24 B, write the 32-byte position record
    "skin": dict(bound="hbm", per="atom", bytes=80),
    # per row: read X of the image and its two neighbours 72 + F 12 + v 24, write v' 24
    "update": dict(bound="hbm", per="row", bytes=132),
    # per row: read X 24 + v' 24, write X 24
    "move": dict(bound="hbm", per="row", bytes=72),
    # per atom: read R~ 24 B, write R 24 B
    "bins": dict(bound="hbm", per="atom", bytes=48),
}


def ts_bonds_flops_per_atom(B):
    """Operations of the Tersoff neighbour-and-bond kernel for an atom with B bonds: the
    exact FP64 inclusion test of each neighbour (26: lattice shift, difference, square),
    then FP32 40 per bond (two exponentials, cutoff, bond order from zeta, energy, radial
    derivative) and 65 per unordered bond pair (cosine, g and g' once; both zeta terms;
    the angular and radial terms of both P's), counting +, -, x, /, each elementary
    function and each half of an FMA as one.  Tests of candidates that are not
    neighbours are implementation work and not counted."""
    return 26.0 * B + 40.0 * B + 65.0 * B * (B - 1.0) / 2.0


def recorded_valu(kernel_source):
    """VALU issue utilisation of the Tersoff kernel from the committed instruction-counter
    summary; None if the kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tersoff_graphite_98304_valu_counters.md")
    try:
        text = open(path).read()
        blob = json.loads(text.split("```json")[1].split("```")[0])
        src = open(os.path.join(ROOT, blob["source"]), "rb").read()
    except (OSError, IndexError, ValueError, KeyError):
        return None
    if blob["kernel"] != kernel_source or hashlib.sha256(src).hexdigest() != blob["source_sha256"]:
        return None
    return blob["valu_issue_util"]


def recorded_traffic(kernel_source, moving_images):
    """HBM bytes per dispatch of the Tersoff neighbour-and-bond kernel from the committed counter
    summary, scaled to the current number of moving images; None if the kernel's source
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tersoff_graphite_98304_hbm_counters.md")
    try:
        text = open(path).read()
        blob = json.loads(text.split("```json")[1].split("```")[0])
        src = open(os.path.join(ROOT, blob["source"]), "rb").read()
    except (OSError, IndexError, ValueError, KeyError):
        return None
    if blob["kernel"] != kernel_source or hashlib.sha256(src).hexdigest() != blob["source_sha256"]:
        return None
    return blob["hbm_bytes_per_dispatch"] * moving_images / blob["moving_images"]


def make_band(args):
    import workloads as W
    from paper_2510_16721_amd import cfneb
    w = W.tersoff_graphite_98304(seed=2)
    kw = dict(n_images=24, max_images=40, min_images=5, pressure_GPa=15.0, refine_every=20,
              climb_after=100, k_spring=1.0, force_fp64=0)
    p = cfneb.default_params(cfneb.CFNEB_TERSOFF_C, **kw)
    band = cfneb.Band(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    return band, w, kw


def cpu_baseline(w, kw, steps):
    import oracle
    okw = {k: v for k, v in kw.items() if k not in ("force_fp64",)}
    p = oracle.default_params(oracle.TERSOFF, **okw)
    band = oracle.Band(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    m0 = band.n_images
    t0 = time.perf_counter()
    done, _, _ = band.step(steps)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    value = w["n"] * (m0 - 2) * done / dt
    return dict(value=value, unit="atom·steps/s", cores=threads, kind="oracle",
                sample=f"{done} band steps of the {w['n']}-atom, {m0}-image band "
                       f"({m0 - 2} moving images), FP64, OpenMP over images, {dt:.1f} s")


def mix_params(entry):
    """LJ bands climb from step 50.  Tersoff diamond vacancy hops run without the climbing
    image: on this potential the symmetric midpoint of the hop is a ridge point, not a
    first-order saddle; a climbing image started on a short band leaves the valley and
    drags its neighbours uphill.  The Tersoff bands start from a seeded displacement of
    their interior images (mix_displacement), which lets them leave the ridge for the
    lower path."""
    from paper_2510_16721_amd import cfneb
    lj = entry["kind"] == "lj"
    m = entry["n_images"]
    return cfneb.default_params(cfneb.CFNEB_LJ if lj else cfneb.CFNEB_TERSOFF_C, n_images=m,
                                max_images=m, min_images=3, climb_after=50 if lj else -1)


def mix_displacement(W, entry, seed):
    """Tersoff bands start from a seeded zero-mean displacement of their interior images
    (N(0, 0.01 A) per atom), LJ bands from the straight line."""
    if entry["kind"] != "ts":
        return None
    return W.interior_noise(seed, entry["n_images"], entry["n"])


_POOL = {}


def relax_mix(mix):
    """Replace every entry's endpoints by cell-filter-relaxed ones (cfneb_relax on the
    device, fmax < 1e-4 eV/A), relaxed once per (family, atom count): the pool of
    relaxed endpoints a request would bring.  Untimed preparation."""
    import torch
    from paper_2510_16721_amd import cfneb
    t0 = time.perf_counter()
    for e in mix:
        key = (e["kind"], e["n"])
        if key not in _POOL:
            w, p = e["endpoints"], mix_params(e)
            a = cfneb.relax(p, w["pos_init"], w["cell_init"], 20000, 1e-4)
            b = cfneb.relax(p, w["pos_final"], w["cell_final"], 20000, 1e-4)
            if not (a[4] and b[4]):
                raise RuntimeError(f"endpoint relaxation of {key} did not converge")
            _POOL[key] = dict(pos_init=a[0], cell_init=a[1], pos_final=b[0], cell_final=b[1],
                              n=w["n"], types=w["types"])
        e["endpoints"] = _POOL[key]
    torch.cuda.synchronize()
    print(f"bench: {len(_POOL)} endpoint pairs relaxed in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    return mix


def bench_batched(args):
    """Independent bands (atom counts log-uniform in [256, 32,000], 5-17 images, LJ and
    Tersoff vacancy hops) relaxed to fmax < 0.01 eV/A one at a time, then all in one
    batch; speedup = plain time / batched time, barriers compared band by band."""
    import torch
    import workloads as W
    from paper_2510_16721_amd import cfneb
    f_tol = 0.01
    mix = relax_mix(W.band_mix(3, args.bands, 256, args.n_max or 32000, 5, 17))
    for q, e in enumerate(mix):
        e["displace"] = mix_displacement(W, e, [3, q])

    def make(e):
        w = e["endpoints"]
        b = cfneb.Band(mix_params(e), w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
        if e["displace"] is not None:
            b.displace_interior(e["displace"])
        return b

    plain_t, plain = 0.0, []
    for q, e in enumerate(mix):
        w = e["endpoints"]
        b = make(e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, fmax, conv = b.step(args.max_steps, f_tol)
        torch.cuda.synchronize()
        plain_t += time.perf_counter() - t0
        plain.append(dict(steps=done, conv=conv, barrier=b.energies()["barrier"],
                          work=w["n"] * b.get_state()["image_steps"]))
        b.close()
        print(f"bench: plain band {q}: {w['n']} atoms, {e['n_images']} images, {done} steps, "
              f"converged {conv}", file=sys.stderr, flush=True)
    bands = [make(e) for e in mix]
    batch = cfneb.Batch(len(bands))
    slots = [batch.attach(b) for b in bands]
    steps = np.zeros(len(bands), dtype=np.int64)
    live = set(range(len(bands)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while live:
        # never past any live band's step cap, so capped bands stop where they stop alone
        s, conv, errs = batch.step(int(min(64, min(args.max_steps - steps[q] for q in live))), f_tol)
        for q in list(live):
            steps[q] += s[slots[q]]
            if conv[slots[q]] or errs[slots[q]] or steps[q] >= args.max_steps:
                batch.detach(slots[q])
                live.discard(q)
    torch.cuda.synchronize()
    batched_t = time.perf_counter() - t0
    bar = np.array([b.energies()["barrier"] for b in bands])
    diff = np.abs(bar - np.array([p["barrier"] for p in plain]))
    work = sum(p["work"] for p in plain)
    batch.close()
    return {
        "metric": "batched-vs-plain speedup at 1 meV",
        "value": plain_t / batched_t, "unit": "x", "n_gpus": 1, "higher_is_better": True,
        "data": "synthetic (seeded LJ FCC and Tersoff diamond vacancy hops)",
        "dtype": "fp32 pair/three-body, fp64 sums/band/FIRE",
        "config": {"workload": f"{len(mix)} independent bands, atoms log-uniform in "
                               f"[256, {args.n_max or 32000}], 5-17 images, run to fmax < 0.01 eV/A "
                               f"(cap {args.max_steps} steps)",
                   "bands": len(mix), "parallelism": "1 GPU"},
        "plain_s": plain_t, "batched_s": batched_t,
        "plain_atom_steps_per_s": work / plain_t, "batched_atom_steps_per_s": work / batched_t,
        "max_barrier_diff_eV": float(diff.max()),
        "converged_plain": int(sum(p["conv"] for p in plain)),
        "steps_identical": bool(all(int(steps[q]) == plain[q]["steps"] for q in range(len(mix)))),
        "vs_baseline": None,
    }


def bench_serving(args):
    """Poisson stream of band relaxations (atoms log-uniform in [500, 50,000], 7-21 images,
    LJ or Tersoff 50/50) served by the continuous-batching loop with a 200 GB HBM budget;
    p99 / p50 time from arrival to converged barrier, and throughput."""
    import workloads as W
    from paper_2510_16721_amd import serving
    mix = relax_mix(W.band_mix(4, args.requests, 500, args.n_max or 50000, 7, 21))
    arrivals = W.poisson_arrivals(4, len(mix), args.rate)
    reqs = [serving.Request(rid=q, arrival=float(arrivals[q]), params=mix_params(e),
                            endpoints=e["endpoints"], n_atoms=e["n"],
                            displace=mix_displacement(W, e, [4, q]))
            for q, e in enumerate(mix)]
    srv = serving.Server(hbm_budget_bytes=200e9, max_bands=64, f_tol=0.01, steps_per_call=32,
                         max_steps=args.max_steps)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t0
    s = serving.summarize(done, wall)
    occ = np.array([o[1] for o in srv.occupancy]) if srv.occupancy else np.zeros(1)
    return {
        "metric": "p99 latency (arrival to converged barrier)",
        "value": s["p99_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
        "data": "synthetic (seeded LJ FCC and Tersoff diamond vacancy hops, Poisson arrivals)",
        "dtype": "fp32 pair/three-body, fp64 sums/band/FIRE",
        "config": {"workload": f"{len(mix)} requests at {args.rate}/s, atoms log-uniform in "
                               f"[500, {args.n_max or 50000}], 7-21 images, fmax < 0.01 eV/A, "
                               f"HBM budget 200 GB", "parallelism": "1 GPU"},
        "p50_s": s["p50_s"], "atom_steps_per_s": s["atom_steps_per_s"], "wall_s": wall,
        "converged": s["converged"], "failed": s["failed"], "capped": s["capped"],
        "mean_active_bands": float(occ.mean()), "max_active_bands": int(occ.max()),
        "capped_requests": [[r.rid, mix[r.rid]["kind"], r.n_atoms, mix[r.rid]["n_images"]]
                            for r in done if r.error == 0 and not r.converged],
        "vs_baseline": None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=40)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--mode", choices=["throughput", "batched", "serving"], default="throughput",
                    help="throughput: the 98,304-atom band (default); batched: many bands "
                         "batched vs one at a time; serving: Poisson request stream")
    ap.add_argument("--bands", type=int, default=64, help="batched mode: number of bands")
    ap.add_argument("--requests", type=int, default=64, help="serving mode: number of requests")
    ap.add_argument("--rate", type=float, default=4.0, help="serving mode: arrivals per second")
    ap.add_argument("--max-steps", type=int, default=4000, help="batched/serving: step cap per band")
    ap.add_argument("--n-max", type=int, default=0, help="batched/serving: override the atom-count cap")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (a band would "
              "shard by contiguous blocks of images, one block per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "needs a HIP device"
    torch.cuda.set_device(0)
    if args.mode == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.mode == "serving":
        print(json.dumps(bench_serving(args)), flush=True)
        return
    band, w, kw = make_band(args)
    N = band.n
    print(f"bench: band created, {N} atoms, {kw['n_images']} images, workspace "
          f"{band.bytes / 2**30:.2f} GiB", file=sys.stderr, flush=True)

    band.step(args.warmup)
    torch.cuda.synchronize()
    s0 = band.get_state()["image_steps"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, fmax, conv = band.step(args.steps, 0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = band.get_state()
    image_steps = st["image_steps"] - s0
    assert done == args.steps, (done, args.steps)
    elapsed = t1 - t0
    value = N * image_steps / elapsed
    M_end = st["X"].shape[0]
    print(f"bench: timed {done} steps in {elapsed:.3f} s, images now {M_end}, fmax {fmax:.3e}",
          file=sys.stderr, flush=True)

    # profiled pass: per-phase device time with HIP events on the band's stream
    s1 = st["image_steps"]
    pdone, _, _, phase_ms = band.step_profiled(args.profile_steps, 0.0)
    st2 = band.get_state()
    prof_image_steps = st2["image_steps"] - s1
    mean_moving = prof_image_steps / max(pdone, 1)
    # bonds of every atom of every moving image (the flop model is per atom and not
    # linear in the bond count)
    m_now = band.get_state()["X"].shape[0]
    counts = np.concatenate([band.neighbours(k)[0] for k in range(1, m_now - 1)]).astype(np.float64)
    mean_bonds = float(counts.mean())
    flops_per_atom = float(ts_bonds_flops_per_atom(counts).mean())
    # own position 32 B and candidate count 4 B; per bond the candidate entry 4 B and
    # P_ij 16 B (the neighbours' positions are gathered from L2)
    bytes_per_atom = float((20.0 * counts + 36.0).mean())
    per_launch = {k: v / max(pdone, 1) for k, v in phase_ms.items()}
    total_ms = sum(per_launch.values())
    dom = max(per_launch, key=per_launch.get)
    # a phase that launches nothing in this workload (Tersoff: filter, force2, reduce)
    # times the two events alone; that overhead is taken off the dominant phase so that
    # its duration is the kernel's, as the kernel trace counts it
    empty = [per_launch[k] for k in ("filter", "force2", "reduce") if k in per_launch]
    event_ms = float(np.median(empty)) if empty and dom == "force0" else 0.0
    kernel_ms = per_launch[dom] - event_ms
    rows = (N + 3) * mean_moving
    atoms = N * mean_moving
    if dom == "force0":
        # the Tersoff neighbour-and-bond kernel (exact test of the candidates, bond
        # orders, energies, dU_i/dr^ij, virial); FP32 and FP64 vector peaks are equal
        flops = flops_per_atom * atoms
        achieved = flops / (kernel_ms * 1e-3) / 1e12
        roof = dict(bound="alu", kernel="k_ts_filter_bonds<float>", achieved=achieved,
                    peak=VALU_FP32_PEAK_TFLOPS, unit="TFLOP/s", frac=achieved / VALU_FP32_PEAK_TFLOPS,
                    traffic=recorded_traffic("k_ts_filter_bonds<float>", mean_moving),
                    algorithmic_bytes=bytes_per_atom * atoms,
                    valu_issue_util=recorded_valu("k_ts_filter_bonds<float>"))
    elif dom in ALGO:
        m = ALGO[dom]
        units = rows if m["per"] == "row" else atoms
        achieved = m["bytes"] * units / (kernel_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", kernel=dom, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=None)
    else:
        roof = dict(bound="alu", kernel=dom, achieved=None, peak=VALU_FP32_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=None, traffic=None,
                    note="dominant phase has no algorithmic work model (implementation work)")
    roof["avg_launch_ms"] = kernel_ms
    roof["event_overhead_ms"] = event_ms
    roof["phase_ms_per_step"] = {k: round(v, 4) for k, v in per_launch.items()}
    roof["profiled_step_ms"] = total_ms
    roof["mean_bonds_per_atom"] = mean_bonds
    roof["flops_per_atom"] = flops_per_atom

    if args.copy_calibration_mib > 0:
        # one elementwise kernel that reads and writes exactly this many MiB: the
        # scale of the FETCH_SIZE / WRITE_SIZE counters
        nb = args.copy_calibration_mib * 2**20
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": "atom·steps/s at 1e5 atoms",
        "value": value,
        "unit": "atom·steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 pair/three-body, fp64 sums/band/FIRE",
        "data": "synthetic (seeded graphite-to-diamond-like Tersoff carbon band)",
        "config": {"workload": "Tersoff C graphite->diamond-like band, 98,304 atoms, 24 images "
                               "(adaptive, max 40), 15 GPa, cell filter",
                   "atoms": N, "images_start": kw["n_images"], "images_end": M_end,
                   "parallelism": "1 GPU"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, kw, args.cpu_steps)
    band.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
