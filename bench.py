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
events around every phase on the band's stream) and "cpu_baseline" (the FP64
oracle on the host cores, on a bounded sample of the same workload).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.
# The kernels are built with packed FP32 disabled, so the unpacked rate is the ceiling.
VALU_FP32_PEAK_TFLOPS = 78.6

# Algorithmic work per unit (documented with the derivations in the design doc).
#   rows = (atoms + 3) per moving image; atoms = atoms per moving image
#   Tersoff flops: 60 per directed bond + 80 per bond pair (triplet) for energy and forces
ALGO = {
    # per row: read X 24 B + F 12 B + v 24 B
    "dots": dict(bound="hbm", per="row", bytes=60),
    # per row: read X 24 + F 12 + v 24, write v' 24
    "update": dict(bound="hbm", per="row", bytes=84),
    # per row: read X 24 + v' 24, write X 24
    "move": dict(bound="hbm", per="row", bytes=72),
    # per atom: read R~ 24 B, write R 24 B
    "bins": dict(bound="hbm", per="atom", bytes=48),
}


def tersoff_flops_per_atom(mean_bonds):
    B = mean_bonds
    return 60.0 * B + 80.0 * B * (B - 1.0)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=40)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the band would shard by contiguous image blocks; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "needs a HIP device"
    torch.cuda.set_device(0)
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
    cnt, _ = band.neighbours(1)
    mean_bonds = float(cnt.mean())
    per_launch = {k: v / max(pdone, 1) for k, v in phase_ms.items()}
    total_ms = sum(per_launch.values())
    dom = max(per_launch, key=per_launch.get)
    rows = (N + 3) * mean_moving
    atoms = N * mean_moving
    if dom in ("force0", "force1", "force2"):
        flops = tersoff_flops_per_atom(mean_bonds) * atoms
        fms = per_launch["force0"] + per_launch["force1"] + per_launch["force2"]
        achieved = flops / (fms * 1e-3) / 1e12
        roof = dict(bound="alu", kernel="tersoff force (3 kernels)", achieved=achieved,
                    peak=VALU_FP32_PEAK_TFLOPS, unit="TFLOP/s", frac=achieved / VALU_FP32_PEAK_TFLOPS,
                    traffic=None)
    elif dom in ALGO:
        m = ALGO[dom]
        units = rows if m["per"] == "row" else atoms
        achieved = m["bytes"] * units / (per_launch[dom] * 1e-3) / 1e9
        roof = dict(bound="hbm", kernel=dom, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=None)
    else:
        roof = dict(bound="alu", kernel=dom, achieved=None, peak=VALU_FP32_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=None, traffic=None,
                    note="dominant phase has no algorithmic work model (implementation work)")
    roof["avg_launch_ms"] = per_launch[dom]
    roof["phase_ms_per_step"] = {k: round(v, 4) for k, v in per_launch.items()}
    roof["profiled_step_ms"] = total_ms
    roof["mean_bonds_per_atom"] = mean_bonds

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib * 2**20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
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
