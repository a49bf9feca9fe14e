"""Benchmark of the CFNEB band step on one MI355X.

Workload: graphite to cubic-diamond-like Tersoff carbon band, 98,304 atoms per
image, 24 initial images (adaptive insertion up to 40, checked every 20 steps),
15 GPa hydrostatic pressure through the rotation-free cell filter, FP32 pair and
three-body arithmetic with FP64 sums, band, cell filter and FIRE in FP64.

A step is one pass of the whole band step (every moving image: geometry, cell
list, neighbour list, forces, virial, cell filter; then tangents, springs,
climbing image, FIRE, and the adaptive-image check).  value = atoms x moving
images x steps / seconds over exactly --steps steps, inputs resident in HBM.

Prints one JSON line.  Beside the throughput it carries:
  roofline      the kernel with the most device time against its bound (HIP events
                around every phase on the band's stream in a second, profiled pass),
                and the phase-summed fraction of the whole step;
  parity        errors of one moving image of the timed band against the FP64 oracle;
  cpu_baseline  the FP64 oracle on the host cores (OpenMP over images, and one thread);
  batched       many independent bands relaxed one at a time and in one batch;
  serving       a Poisson stream of band relaxations through the request loop.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak of MI355X without packed math: 256 CUs x 4 SIMD x 16 lanes x 2 flop
# (FMA) x 2.4 GHz.  The kernels are built with packed FP32 disabled, so this is the
# ceiling; the packed figure is reported beside it.
VALU_FP32_PEAK_TFLOPS = 78.6
VALU_FP32_PACKED_PEAK_TFLOPS = 157.3
# algorithmic HBM bytes of the band, cell-filter and FIRE passes per atom (row) per
# moving image per step: read R~ 24, write the generalized force 24, the dots pass
# (X, force, v) 72, the update passes (X, force, v in; v, X out) 120
BAND_BYTES_PER_ROW = 240.0

# Algorithmic work per unit of the streaming phases (bytes that must cross HBM once).
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

TOL = dict(E_per_atom=1e-6, F=1e-4, V_per_atom=1e-5)


def ts_flops_per_atom(B):
    """Algorithmic FP32 work of the Tersoff energy and forces for an atom with B bonds:
    about 60 operations per directed bond (two exponentials, cutoff, bond order, radial
    terms) and 80 per ordered bond pair, of which there are B (B - 1) (angle, g, g',
    zeta terms and the three-body forces); transcendentals count as 4."""
    return 60.0 * B + 80.0 * B * (B - 1.0)


def source_fingerprint():
    """sha256 over every HIP source and header of the library and its build flags: a
    recorded counter figure belongs to exactly this build."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2510_16721_amd")
    files = sorted(glob.glob(os.path.join(pkg, "csrc", "*.hip")) + glob.glob(os.path.join(pkg, "csrc", "*.h")))
    files += [os.path.join(ROOT, "include", "cfneb.h"), os.path.join(pkg, "build.py")]
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def recorded(summary, key, scale_images=None):
    """A figure of a committed counter summary (profiles/), or None when the library's
    sources or build flags changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        text = open(path).read()
        blob = json.loads(text.split("```json")[1].split("```")[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("fingerprint") != source_fingerprint() or key not in blob:
        return None
    v = blob[key]
    if scale_images is not None:
        v = v * scale_images / blob["moving_images"]
    return v


def make_band(potential):
    import workloads as W
    from paper_2510_16721_amd import cfneb
    kw = dict(n_images=24, max_images=40, min_images=5, refine_every=20, climb_after=100, k_spring=1.0,
              force_fp64=0)
    if potential == "tersoff":
        w = W.tersoff_graphite_98304(seed=2)
        kw["pressure_GPa"] = 15.0
        p = cfneb.default_params(cfneb.CFNEB_TERSOFF_C, **kw)
    else:
        w = W.fcc_vacancy_hop(29, 29, 29, 1.5496)  # 97,555 atoms
        p = cfneb.default_params(cfneb.CFNEB_LJ, **kw)
    band = cfneb.Band(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    return band, w, kw


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, kw, potential, steps, single_steps):
    """The oracle as it stands on the host cores: OpenMP over images for `steps` band
    steps, then one thread for `single_steps` steps of the same band."""
    import oracle
    okw = {k: v for k, v in kw.items() if k not in ("force_fp64",)}
    p = oracle.default_params(oracle.TERSOFF if potential == "tersoff" else oracle.LJ, **okw)
    band = oracle.Band(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    m0 = band.n_images
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    done, _, _ = band.step(steps)
    dt = time.perf_counter() - t0
    value = w["n"] * (m0 - 2) * done / dt
    out = dict(value=value, unit="atom·steps/s", cores=threads, kind="oracle",
               sample=f"{done} band steps of the {w['n']}-atom, {m0}-image band ({m0 - 2} moving "
                      f"images), FP64, OpenMP over images on {threads} threads, {dt:.1f} s",
               cpu_model=cpu_model(), nproc=os.cpu_count())
    if single_steps > 0:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        d1, _, _ = band.step(single_steps)
        dt1 = time.perf_counter() - t0
        oracle.set_threads(threads)
        out["single_thread"] = dict(value=w["n"] * (band.n_images - 2) * d1 / dt1, cores=1,
                                    sample=f"{d1} further steps of the same band on one thread, {dt1:.1f} s")
    return out


def parity_sample(band, kw, potential):
    """Per-result errors of one moving image of the band against the oracle, evaluated
    from the device's own positions and cell (the band is evaluated without a move)."""
    import oracle
    band.step(1, 1e30)  # evaluate every moving image; f_tol 1e30 converges without moving
    M = band.get_state()["X"].shape[0]
    k = M // 2
    img = band.image(k)
    okw = {k2: v for k2, v in kw.items() if k2 not in ("force_fp64",)}
    p = oracle.default_params(oracle.TERSOFF if potential == "tersoff" else oracle.LJ, **okw)
    t0 = time.perf_counter()
    E, u, F, V = oracle.evaluate(p, img["R"], img["h"])
    n = band.n
    out = dict(image=k, atoms=n,
               E_err_per_atom=abs(img["E"] - E) / n,
               F_err_max=float(np.abs(img["F"] - F).max()),
               V_err_per_atom=float(np.abs(img["V"] - V).max() / n),
               tolerances=TOL, oracle_s=round(time.perf_counter() - t0, 2))
    out["within"] = bool(out["E_err_per_atom"] <= TOL["E_per_atom"] and out["F_err_max"] <= TOL["F"]
                         and out["V_err_per_atom"] <= TOL["V_per_atom"])
    return out


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


def bench_batched(bands, max_steps, n_max=0):
    """Independent bands (atom counts log-uniform in [256, 32,000], 5-17 images, LJ and
    Tersoff vacancy hops) relaxed to fmax < 0.01 eV/A one at a time, then all in one
    batch; speedup = plain time / batched time over the steps alone (every band's and
    the batch's graphs are captured before the clocks start), barriers compared band by
    band."""
    import torch
    import workloads as W
    from paper_2510_16721_amd import cfneb
    f_tol = 0.01
    mix = relax_mix(W.band_mix(3, bands, 256, n_max or 32000, 5, 17))
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
        b.step(0)  # force-grid tuning and graph capture, outside the clock
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, fmax, conv = b.step(max_steps, f_tol)
        torch.cuda.synchronize()
        plain_t += time.perf_counter() - t0
        plain.append(dict(steps=done, conv=conv, barrier=b.energies()["barrier"],
                          work=w["n"] * b.get_state()["image_steps"]))
        b.close()
    bands_ = [make(e) for e in mix]
    batch = cfneb.Batch(len(bands_))
    slots = [batch.attach(b) for b in bands_]
    batch.step(0)  # tuning and capture of the batch's graphs, outside the clock
    steps = np.zeros(len(bands_), dtype=np.int64)
    live = set(range(len(bands_)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while live:
        # never past any live band's step cap, so capped bands stop where they stop alone
        s, conv, errs = batch.step(int(min(64, min(max_steps - steps[q] for q in live))), f_tol)
        for q in list(live):
            steps[q] += s[slots[q]]
            if conv[slots[q]] or errs[slots[q]] or steps[q] >= max_steps:
                batch.detach(slots[q])
                live.discard(q)
    torch.cuda.synchronize()
    batched_t = time.perf_counter() - t0
    bar = np.array([b.energies()["barrier"] for b in bands_])
    diff = np.abs(bar - np.array([p["barrier"] for p in plain]))
    work = sum(p["work"] for p in plain)
    batch.close()
    for b in bands_:
        b.close()
    return {
        "metric": "batched-vs-plain speedup at 1 meV",
        "value": plain_t / batched_t, "unit": "x",
        "workload": f"{len(mix)} independent bands, atoms log-uniform in [256, {n_max or 32000}], "
                    f"5-17 images, LJ and Tersoff vacancy hops, run to fmax < 0.01 eV/A (cap {max_steps} steps)",
        "plain_s": plain_t, "batched_s": batched_t,
        "plain_atom_steps_per_s": work / plain_t, "batched_atom_steps_per_s": work / batched_t,
        "max_barrier_diff_eV": float(diff.max()),
        "bands_within_1meV": int((diff <= 1e-3).sum()),
        "converged_plain": int(sum(p["conv"] for p in plain)),
        "capped": int(sum(1 for p in plain if not p["conv"])),
        "steps_identical": bool(all(int(steps[q]) == plain[q]["steps"] for q in range(len(mix)))),
    }


def bench_serving(requests, rate, max_steps, n_max=0, rate_fraction=0.7):
    """Poisson stream of band relaxations (atoms log-uniform in [500, 50,000] from 32 size
    classes per family, 7-21 images, LJ or Tersoff 50/50) served by the continuous-
    batching loop with a 200 GB HBM budget.  rate <= 0: the arrival rate is
    rate_fraction of the loop's capacity, measured first by serving the same requests
    all arriving at once (requests per second at saturation)."""
    import workloads as W
    from paper_2510_16721_amd import serving
    mix = relax_mix(W.band_mix(4, requests, 500, n_max or 50000, 7, 21, size_classes=32))

    def reqs(arrivals):
        return [serving.Request(rid=q, arrival=float(arrivals[q]), params=mix_params(e),
                                endpoints=e["endpoints"], n_atoms=e["n"],
                                displace=mix_displacement(W, e, [4, q]))
                for q, e in enumerate(mix)]

    def server():
        return serving.Server(hbm_budget_bytes=200e9, max_bands=64, f_tol=0.01, steps_per_call=32,
                              max_steps=max_steps)

    capacity = None
    if rate <= 0:
        srv = server()
        t0 = time.perf_counter()
        srv.run(reqs(np.zeros(len(mix))))
        sat = time.perf_counter() - t0
        capacity = len(mix) / sat
        rate = rate_fraction * capacity
        print(f"bench: serving capacity {capacity:.1f} requests/s (all {len(mix)} at once in {sat:.1f} s); "
              f"arrival rate {rate:.1f}/s", file=sys.stderr, flush=True)
    srv = server()
    t0 = time.perf_counter()
    done = srv.run(reqs(W.poisson_arrivals(4, len(mix), rate)))
    wall = time.perf_counter() - t0
    s = serving.summarize(done, wall)
    occ = np.array([o[1] for o in srv.occupancy]) if srv.occupancy else np.zeros(1)
    return {
        "metric": "p99 latency (arrival to converged barrier)",
        "value": s["p99_s"], "unit": "s",
        "workload": f"{len(mix)} requests, Poisson arrivals at {rate:.2f}/s, atoms log-uniform in "
                    f"[500, {n_max or 50000}] (32 size classes per family), 7-21 images, "
                    f"fmax < 0.01 eV/A (cap {max_steps} steps), HBM budget 200 GB",
        "p50_s": s["p50_s"], "p99_converged_s": s["p99_converged_s"], "p50_converged_s": s["p50_converged_s"],
        "percentiles_over": "every request; a capped or failed request at its time to that end",
        "rate_per_s": rate, "capacity_per_s": capacity,
        "atom_steps_per_s": s["atom_steps_per_s"], "wall_s": wall,
        "converged": s["converged"], "failed": s["failed"], "capped": s["capped"],
        "mean_active_bands": float(occ.mean()), "max_active_bands": int(occ.max()),
        "capped_requests": [[r.rid, mix[r.rid]["kind"], r.n_atoms, mix[r.rid]["n_images"]]
                            for r in done if r.error == 0 and not r.converged],
    }


def throughput(args):
    import torch
    band, w, kw = make_band(args.potential)
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
    mean_moving_timed = image_steps / args.steps
    print(f"bench: timed {done} steps in {elapsed:.3f} s, images now {M_end}, fmax {fmax:.3e}",
          file=sys.stderr, flush=True)

    # profiled pass: per-phase device time with HIP events on the band's stream
    s1 = st["image_steps"]
    pdone, _, _, phase_ms = band.step_profiled(args.profile_steps, 0.0)
    st2 = band.get_state()
    prof_image_steps = st2["image_steps"] - s1
    mean_moving = prof_image_steps / max(pdone, 1)
    per_launch = {k: v / max(pdone, 1) for k, v in phase_ms.items()}
    total_ms = sum(per_launch.values())
    dom = max(per_launch, key=per_launch.get)
    # a phase that launches nothing in this workload times the two events alone; that
    # overhead is taken off the dominant phase so that its duration is the kernel's, as
    # the kernel trace counts it
    empty_phases = ("filter", "force2", "reduce") if args.potential == "tersoff" else ("force1", "force2",
                                                                                        "reduce")
    empty = [per_launch[k] for k in empty_phases if k in per_launch]
    event_ms = float(np.median(empty)) if empty else 0.0
    kernel_ms = per_launch[dom] - event_ms
    rows = (N + 3) * mean_moving
    atoms = N * mean_moving
    # bonds of every atom of every moving image (the flop model is per atom and not
    # linear in the bond count)
    m_now = st2["X"].shape[0]
    counts = np.concatenate([band.neighbours(k)[0] for k in range(1, m_now - 1)]).astype(np.float64)
    mean_bonds = float(counts.mean())
    fp = source_fingerprint()
    if args.potential == "tersoff":
        flops_per_atom = float(ts_flops_per_atom(counts).mean())
    else:
        # unique pairs (half the neighbours) x about 22 operations
        flops_per_atom = 0.5 * mean_bonds * 22.0
    if dom == "force0" and args.potential == "tersoff":
        # the Tersoff neighbour-and-bond kernel (exact test of the candidates, bond
        # orders, energies, dU_i/dr^ij, virial); FP32 and FP64 vector peaks are equal
        achieved = flops_per_atom * atoms / (kernel_ms * 1e-3) / 1e12
        roof = dict(bound="alu", kernel="k_ts_filter_bonds<float>", achieved=achieved,
                    peak=VALU_FP32_PEAK_TFLOPS, unit="TFLOP/s", frac=achieved / VALU_FP32_PEAK_TFLOPS,
                    frac_of_packed_peak=achieved / VALU_FP32_PACKED_PEAK_TFLOPS,
                    traffic=recorded("tersoff_graphite_98304_hbm_counters.md", "bonds_kernel_hbm_bytes",
                                     mean_moving),
                    algorithmic_bytes=float((20.0 * counts + 36.0).mean()) * atoms,
                    valu_issue_util=recorded("tersoff_graphite_98304_valu_counters.md", "valu_issue_util"))
    elif dom == "force0":
        # the LJ candidate kernel (exact test and pair term of every candidate)
        achieved = flops_per_atom * atoms / (kernel_ms * 1e-3) / 1e12
        roof = dict(bound="alu", kernel="k_lj_cand<float, 1>", achieved=achieved, peak=VALU_FP32_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=achieved / VALU_FP32_PEAK_TFLOPS,
                    traffic=recorded("lj_fcc_vacancy_97555_hbm_counters.md", "force_kernel_hbm_bytes", mean_moving),
                    valu_issue_util=recorded("lj_fcc_vacancy_97555_valu_counters.md", "valu_issue_util"))
    elif dom in ALGO:
        m = ALGO[dom]
        units = rows if m["per"] == "row" else atoms
        achieved = m["bytes"] * units / (kernel_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", kernel=dom, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=None)
    else:
        achieved = flops_per_atom * atoms / (kernel_ms * 1e-3) / 1e12
        roof = dict(bound="alu", kernel=dom, achieved=achieved, peak=VALU_FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=achieved / VALU_FP32_PEAK_TFLOPS, traffic=None)
    roof["avg_launch_ms"] = kernel_ms
    roof["event_overhead_ms"] = event_ms
    roof["phase_ms_per_step"] = {k: round(v, 4) for k, v in per_launch.items()}
    roof["profiled_step_ms"] = total_ms
    roof["mean_bonds_per_atom"] = mean_bonds
    roof["flops_per_atom"] = flops_per_atom
    roof["source_fingerprint"] = fp[:16]
    # phase-summed fraction of the step: force phase at the VALU peak plus the band,
    # cell-filter and FIRE passes at the HBM peak, against the measured step
    t_valu = flops_per_atom * N * mean_moving_timed / (VALU_FP32_PEAK_TFLOPS * 1e12) * 1e3
    t_hbm = BAND_BYTES_PER_ROW * (N + 3) * mean_moving_timed / (HBM_PEAK_GBS * 1e9) * 1e3
    step_ms = elapsed / args.steps * 1e3
    roof["step"] = dict(t_valu_ms=t_valu, t_hbm_ms=t_hbm, bound_ms=t_valu + t_hbm, measured_ms=step_ms,
                        frac=(t_valu + t_hbm) / step_ms)

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

    name = ("Tersoff C graphite->diamond-like band, 98,304 atoms, 24 images (adaptive, max 40), 15 GPa, "
            "cell filter" if args.potential == "tersoff" else
            "LJ FCC vacancy hop, 97,555 atoms, 24 images (adaptive, max 40), cell filter")
    out = {
        "metric": "atom·steps/s at 1e5 atoms",
        "value": value,
        "unit": "atom·steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 pair/three-body, fp64 sums/band/FIRE",
        "data": "synthetic (seeded graphite-to-diamond-like Tersoff carbon band)" if args.potential == "tersoff"
                else "synthetic (LJ FCC vacancy hop)",
        "config": {"workload": name, "atoms": N, "images_start": kw["n_images"], "images_end": M_end,
                   "parallelism": "1 GPU"},
        "roofline": roof,
    }
    if not args.no_parity:
        out["parity"] = parity_sample(band, kw, args.potential)
        print(f"bench: parity sample {out['parity']}", file=sys.stderr, flush=True)
    band.close()
    del band
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, kw, args.potential, args.cpu_steps, args.cpu_single_steps)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=40)
    ap.add_argument("--potential", choices=["tersoff", "lj"], default="tersoff",
                    help="throughput workload: the Tersoff band (default) or a 97,555-atom LJ band")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--cpu-single-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--mode", choices=["all", "throughput", "batched", "serving"], default="all",
                    help="all: throughput line with the batched and serving objects (default)")
    ap.add_argument("--bands", type=int, default=64, help="batched: number of bands")
    ap.add_argument("--requests", type=int, default=500, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serving: arrivals per second (0: 0.7 of the measured capacity)")
    ap.add_argument("--max-steps", type=int, default=10000, help="batched/serving: step cap per band")
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
        print(json.dumps(bench_batched(args.bands, args.max_steps, args.n_max)), flush=True)
        return
    if args.mode == "serving":
        print(json.dumps(bench_serving(args.requests, args.rate, args.max_steps, args.n_max)), flush=True)
        return
    out = throughput(args)
    if args.mode == "all":
        print("bench: batched bands", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(args.bands, args.max_steps, args.n_max)
        print(f"bench: batched {out['batched']['value']:.2f}x", file=sys.stderr, flush=True)
        print("bench: serving", file=sys.stderr, flush=True)
        out["serving"] = bench_serving(args.requests, args.rate, args.max_steps, args.n_max)
        print(f"bench: serving p99 {out['serving']['value']:.2f} s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
