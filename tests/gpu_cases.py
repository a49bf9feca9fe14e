"""Shared builders for the GPU parity tests: the same workload and parameters
handed to the HIP library and to the oracle."""
import numpy as np

import workloads as W

# tolerances of the FP32 force path against the FP64 oracle
TOL_E_PER_ATOM = 1e-6     # eV / atom
TOL_F = 1e-4              # eV / A, max abs
TOL_V_PER_ATOM = 1e-5     # eV / atom / component
TOL_BARRIER = 1e-3        # eV


def workload(name):
    if name == "lj255":
        return W.lj_fcc_hop_255(), "lj"
    if name == "lj31":
        return W.fcc_vacancy_hop(2, 2, 2, 1.5496), "lj"
    if name == "lj_ragged":
        return W.fcc_vacancy_hop(5, 4, 4, 1.5496), "lj"  # 319 atoms: two tiles, ragged tail
    if name == "lj863":
        # 6x6x6 cells: every perpendicular width is above twice rc + 2 skin, so the FP32
        # force kernel takes fixed-point separations; 863 atoms = 3 tiles + 95
        return W.fcc_vacancy_hop(6, 6, 6, 1.5496), "lj"
    if name == "lj863_sheared":
        # the same lattice and cells under a shear (off-diagonal cell entries, a
        # triclinic cell): the 3x3 product of the fixed-point separations
        w = W.fcc_vacancy_hop(6, 6, 6, 1.5496)
        S = np.array([[1.0, 0.08, -0.05], [0.0, 1.0, 0.11], [0.0, 0.0, 1.0]])
        w = dict(w)
        for k in ("pos_init", "pos_final", "cell_init", "cell_final"):
            w[k] = w[k] @ S
        return w, "lj"
    if name == "ts_small":
        return W.small_graphite(), "ts"
    if name == "ts_diamond":
        return W.diamond_vacancy_hop(2, 2, 2), "ts"
    if name == "ts_dense":
        # random carbon at 0.2 atoms/A^3: most atoms have more than 6 bonds inside 2.1 A
        R, h = W.random_cell(160, 21, density=0.2, skew=0.2, min_sep=1.1)
        return dict(pos_init=R, cell_init=h, pos_final=R.copy(), cell_final=h * 1.02,
                    n=len(R)), "ts"
    if name == "ts4608":
        return W.tersoff_graphite_4608(), "ts"
    if name == "ts98304":
        return W.tersoff_graphite_98304(), "ts"
    raise KeyError(name)


# parameters of the device's data structures only (no effect on the results)
DEVICE_ONLY = ("nbr_cap", "nbr_skin")


def make_pair(name, fp64=False, oracle_too=True, **kw):
    import oracle
    from paper_2510_16721_amd import cfneb
    w, kind = workload(name)
    gp = cfneb.default_params(cfneb.CFNEB_LJ if kind == "lj" else cfneb.CFNEB_TERSOFF_C,
                              force_fp64=1 if fp64 else 0, **kw)
    g = cfneb.Band(gp, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    o = None
    if oracle_too:
        op = oracle.default_params(oracle.LJ if kind == "lj" else oracle.TERSOFF,
                                   **{k: v for k, v in kw.items() if k not in DEVICE_ONLY})
        o = oracle.Band(op, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    return g, o, w, kind


def oracle_params_like(kind, **kw):
    import oracle
    return oracle.default_params(oracle.LJ if kind == "lj" else oracle.TERSOFF,
                                 **{k: v for k, v in kw.items() if k not in DEVICE_ONLY})


def sort_entries(ent):
    if len(ent) == 0:
        return ent.reshape(0, 4)
    order = np.lexsort((ent[:, 3], ent[:, 2], ent[:, 1], ent[:, 0]))
    return ent[order]
