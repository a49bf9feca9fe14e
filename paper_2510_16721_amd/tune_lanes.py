"""Autotuner of the LJ force kernel's lanes per atom (1, 2, 4 or 8 lanes of a
wavefront share one atom's candidates).

For LJ FCC vacancy-hop bands over a range of sizes (atoms x images), each lane
count is timed on the band stepped alone (HIP-event phase timing of the force
stage, cfneb_step_profiled); the fastest count per size becomes a row of
csrc/lj_lanes_table.h, which the library compiles in and looks up at band
creation.  A band keeps its count alone and in a batch, so a batch never changes
its sums.

    python -m paper_2510_16721_amd.tune_lanes            # measure and print
    python -m paper_2510_16721_amd.tune_lanes --write    # and rewrite the table
(then rebuild the library).
"""
import argparse
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "lj_lanes_table.h")
LANES = (1, 2, 4, 8)
# (FCC cells per edge, images): 31 .. 97,555 atoms, 217 .. 2.3M atom-images
CASES = [(2, 7), (3, 7), (4, 7), (6, 7), (8, 7), (11, 7), (16, 7), (22, 7), (29, 7), (29, 24)]


def _band(n, images):
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads as W
    from . import cfneb
    w = W.fcc_vacancy_hop(n, n, n, 1.5496)
    p = cfneb.default_params(cfneb.CFNEB_LJ, n_images=images, max_images=images, climb_after=-1)
    return cfneb.Band(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"]), w["n"]


def time_case(n, images, steps=20, warmup=5):
    """Force-stage ms per step for each lane count."""
    out = {}
    for k in LANES:
        os.environ["CFNEB_LJ_LANES"] = str(k)
        try:
            band, atoms = _band(n, images)
            band.step(warmup)
            _, _, _, ph = band.step_profiled(steps)
            out[k] = ph["force0"] / steps
            band.close()
        finally:
            del os.environ["CFNEB_LJ_LANES"]
    return atoms, out


def pick(t, margin=0.03):
    """The fewest lanes within `margin` of the fastest time (ties and timing noise keep
    the simpler shape)."""
    best = min(t.values())
    return min(k for k in t if t[k] <= best * (1.0 + margin))


def table_rows(results):
    """results: [(atom_images, {lanes: ms})] -> [(max_atom_images, lanes)], thresholds at
    the geometric mean of neighbouring sizes whose picked counts differ."""
    pts = sorted((w, pick(t)) for w, t in results)
    rows = []
    for i, (w, k) in enumerate(pts):
        if i + 1 < len(pts) and pts[i + 1][1] == k:
            continue
        if i + 1 < len(pts):
            rows.append((int(math.sqrt(w * pts[i + 1][0])), k))
        else:
            rows.append((None, k))
    return rows


def write_table(rows, results, path=TABLE):
    lines = ["// LJ lanes per atom by band size (atoms x images at creation): the fastest lane",
             "// count of an FP32 LJ band stepped alone.  Written by tune_lanes.py from",
             "// force-stage times (us per step) of LJ FCC vacancy-hop bands:"]
    for w, t in sorted(results):
        lines.append("//   " + f"{w:>9d} atom-images: " +
                     "  ".join(f"{k}: {1000 * t[k]:8.1f}" for k in LANES))
    lines += ["#ifndef CFNEB_LJ_LANES_TABLE_H", "#define CFNEB_LJ_LANES_TABLE_H", "",
              "struct LjLanesEntry {", "    long long max_atom_images;", "    int lanes;", "};",
              "static const LjLanesEntry kLjLanesTable[] = {"]
    for w, k in rows:
        lines.append(f"    {{{w if w is not None else 9223372036854775807}LL, {k}}},")
    lines += ["};", "", "#endif", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--write", action="store_true", help="rewrite csrc/lj_lanes_table.h")
    ap.add_argument("--out", default=TABLE, help="where --write puts the table")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("tune_lanes: needs a HIP device")
    results = []
    for n, images in CASES:
        atoms, t = time_case(n, images)
        results.append((atoms * images, t))
        print(f"tune_lanes: {atoms} atoms x {images} images: " +
              "  ".join(f"K={k} {1000 * t[k]:.1f} us" for k in LANES), flush=True)
    rows = table_rows(results)
    print("tune_lanes: table", rows, flush=True)
    if args.write:
        write_table(rows, results, args.out)
        print(f"tune_lanes: wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
