"""FP64 CPU oracle of the CFNEB band step -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the CPU-baseline leg of the benchmark may use
this package.  The HIP library never imports, links or calls it, and the two
share no code.  See oracle.h for what each function follows in the paper
(arXiv:2510.16721) and how it is pinned.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

LJ = 1
TERSOFF = 2

OK, EINVAL, ECELL, ENEIGH, ENONFINITE, ERANGE = 0, -1, -4, -5, -6, -8


class Params(ctypes.Structure):
    _fields_ = [
        ("potential", ctypes.c_int),
        ("lj_eps", ctypes.c_double), ("lj_sigma", ctypes.c_double), ("lj_rc", ctypes.c_double),
        ("lj_shift", ctypes.c_int),
        ("ts_A", ctypes.c_double), ("ts_B", ctypes.c_double),
        ("ts_lambda1", ctypes.c_double), ("ts_lambda2", ctypes.c_double),
        ("ts_beta", ctypes.c_double), ("ts_n", ctypes.c_double),
        ("ts_c", ctypes.c_double), ("ts_d", ctypes.c_double), ("ts_h", ctypes.c_double),
        ("ts_R", ctypes.c_double), ("ts_S", ctypes.c_double),
        ("n_images", ctypes.c_int), ("max_images", ctypes.c_int), ("min_images", ctypes.c_int),
        ("k_spring", ctypes.c_double), ("climb_after", ctypes.c_int),
        ("cell_filter", ctypes.c_int), ("cell_factor", ctypes.c_double),
        ("b_force_scale", ctypes.c_double), ("pressure_GPa", ctypes.c_double),
        ("fire_dt0", ctypes.c_double), ("fire_dtmax", ctypes.c_double),
        ("fire_maxstep", ctypes.c_double), ("fire_nmin", ctypes.c_int),
        ("fire_finc", ctypes.c_double), ("fire_fdec", ctypes.c_double),
        ("fire_astart", ctypes.c_double), ("fire_fa", ctypes.c_double),
        ("refine_every", ctypes.c_int),
        ("ins_num", ctypes.c_int), ("ins_den", ctypes.c_int),
        ("del_num", ctypes.c_int), ("del_den", ctypes.c_int),
        ("stress_GPa", ctypes.c_double * 6),
    ]


class FireState(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("alpha", ctypes.c_double), ("n_pos", ctypes.c_int),
                ("fresh", ctypes.c_int), ("step", ctypes.c_int), ("ci", ctypes.c_int)]


def lib():
    """Load liborc.so, building it first if it is missing."""
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _LIB = ctypes.CDLL(path)
        _declare(_LIB)
    return _LIB


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def _declare(L):
    c_int, c_double, c_int64, c_void = ctypes.c_int, ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
    L.orc_det3.restype = c_double
    L.orc_det3.argtypes = [_dp]
    L.orc_inv3.argtypes = [_dp, _dp]
    L.orc_symsqrt.argtypes = [_dp, _dp]
    L.orc_widths.argtypes = [_dp, _dp]
    for f in (L.orc_nlist_brute, L.orc_nlist_cells):
        f.restype = c_int64
        f.argtypes = [c_int, _dp, _dp, c_double, _ip, _ip, c_int64]
    L.orc_eval.argtypes = [ctypes.POINTER(Params), c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_cf_eval.argtypes = [ctypes.POINTER(Params), c_int, _dp, _dp, _dp, _dp, _dp, _dp,
                              _dp, _dp, _dp]
    L.orc_build_endpoints.argtypes = [ctypes.POINTER(Params), c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_band_create.restype = c_void
    L.orc_band_create.argtypes = [ctypes.POINTER(Params), c_int, _ip, _dp, _dp, _dp, _dp,
                                  ctypes.POINTER(c_int)]
    L.orc_band_step.argtypes = [c_void, c_int, c_double, ctypes.POINTER(c_int), _dp,
                                ctypes.POINTER(c_int)]
    L.orc_band_refine.argtypes = [c_void, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    L.orc_band_energies.argtypes = [c_void, _dp, c_int, ctypes.POINTER(c_int), _dp,
                                    ctypes.POINTER(c_int), _dp]
    L.orc_band_n_images.argtypes = [c_void]
    L.orc_band_get_state.argtypes = [c_void, _dp, _dp, c_int, ctypes.POINTER(FireState), _dp]
    L.orc_band_set_state.argtypes = [c_void, c_int, _dp, _dp, ctypes.POINTER(FireState)]
    L.orc_band_image.argtypes = [c_void, c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_band_destroy.argtypes = [c_void]
    L.orc_profile.argtypes = [c_int, c_int, c_int, _dp, _dp, _dp, _dp, _dp]
    L.orc_spline_eval.argtypes = [c_int, _dp, _dp, _dp, c_int, _dp, _dp]
    L.orc_spline_max.argtypes = [c_int, _dp, _dp, _dp, _dp, _dp]
    L.orc_band_profile.argtypes = [c_void, c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_band_destroy.restype = None
    L.orc_tangent_coeffs.argtypes = [c_double, c_double, c_double, _dp, _dp]
    L.orc_tangent_coeffs.restype = None
    L.orc_refine_decide.argtypes = [c_int, c_int, _dp, c_int, c_int, c_int, c_int, c_int, c_int,
                                    c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int), _dp]
    L.orc_neb2d.argtypes = [c_double, c_int, _dp, c_double, c_int, c_double, c_double, c_double,
                            c_int, c_double, _dp, ctypes.POINTER(c_int), _dp]
    L.orc_relax.argtypes = [ctypes.POINTER(Params), c_int, _dp, _dp, c_int, c_double,
                            ctypes.POINTER(c_int), _dp]
    L.orc_path_coord.argtypes = [c_int, c_int, c_int, _dp, _dp]
    L.orc_set_threads.argtypes = [c_int]
    L.orc_set_threads.restype = None
    L.orc_max_threads.argtypes = []
    L.orc_max_threads.restype = c_int
    L.orc_fire_step.argtypes = [c_int, c_int, c_int, _dp, _dp, _dp, ctypes.POINTER(FireState),
                                c_double, c_double, c_int, c_double, c_double, c_double, c_double]


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def _check(code, what):
    if code != OK:
        raise OracleError(code, what)


# ---------------------------------------------------------------- parameters
TERSOFF_C_1988 = dict(ts_A=1393.6, ts_B=346.74, ts_lambda1=3.4879, ts_lambda2=2.2119,
                      ts_beta=1.5724e-7, ts_n=0.72751, ts_c=38049.0, ts_d=4.3484,
                      ts_h=-0.57058, ts_R=1.8, ts_S=2.1)


def default_params(potential, **kw):
    p = Params()
    p.potential = potential
    p.lj_eps, p.lj_sigma, p.lj_rc, p.lj_shift = 1.0, 1.0, 2.5, 1
    for k, v in TERSOFF_C_1988.items():
        setattr(p, k, v)
    p.n_images, p.max_images, p.min_images = 7, 7, 3
    p.k_spring, p.climb_after = 1.0, 50
    p.cell_filter, p.cell_factor, p.b_force_scale, p.pressure_GPa = 2, 0.0, 1.0, 0.0
    if potential == LJ:
        p.fire_dt0, p.fire_maxstep = 0.005, 0.1
    else:
        p.fire_dt0, p.fire_maxstep = 0.05, 0.1
    p.fire_dtmax = 10.0 * p.fire_dt0
    p.fire_nmin, p.fire_finc, p.fire_fdec, p.fire_astart, p.fire_fa = 5, 1.1, 0.5, 0.1, 0.99
    p.refine_every = 0
    p.ins_num, p.ins_den, p.del_num, p.del_den = 9, 4, 1, 4
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    if "fire_dt0" in kw and "fire_dtmax" not in kw:
        p.fire_dtmax = 10.0 * p.fire_dt0
    return p


# ---------------------------------------------------------------- geometry
def det3(A):
    return lib().orc_det3(_d(_f64(A, 9)))


def inv3(A):
    out = np.zeros(9)
    lib().orc_inv3(_d(_f64(A, 9)), _d(out))
    return out.reshape(3, 3)


def symsqrt(B):
    out = np.zeros(9)
    _check(lib().orc_symsqrt(_d(_f64(B, 9)), _d(out)), "symsqrt")
    return out.reshape(3, 3)


def widths(h):
    out = np.zeros(3)
    lib().orc_widths(_d(_f64(h, 9)), _d(out))
    return out


def nlist(R, h, rc, method="cells"):
    """Per-atom sorted neighbour entries: list of (k, 4) int32 arrays of (j, n0, n1, n2)."""
    R = _f64(R, (-1, 3))
    n = R.shape[0]
    cnt = np.zeros(n, dtype=np.int32)
    f = lib().orc_nlist_cells if method == "cells" else lib().orc_nlist_brute
    cap = max(16, 64 * n)
    while True:
        ent = np.zeros((cap, 4), dtype=np.int32)
        tot = f(n, _d(R), _d(_f64(h, 9)), float(rc), _i(cnt), _i(ent), cap)
        if tot == ECELL:
            raise OracleError(ECELL, "nlist")
        if tot >= 0:
            break
        cap = -tot
    off = np.concatenate([[0], np.cumsum(cnt)])
    return [ent[off[i]:off[i + 1]].copy() for i in range(n)]


def evaluate(p, R, h):
    """E, per-atom u, F (n x 3), V (3 x 3) of positions R in cell h."""
    R = _f64(R, (-1, 3))
    n = R.shape[0]
    E = np.zeros(1)
    u = np.zeros(n)
    F = np.zeros((n, 3))
    V = np.zeros(9)
    _check(lib().orc_eval(ctypes.byref(p), n, _d(R), _d(_f64(h, 9)), _d(E), _d(u), _d(F), _d(V)),
           "eval")
    return E[0], u, F, V.reshape(3, 3)


def cf_eval(p, h0, X):
    """One image through the cell filter.  X is (n+3) x 3."""
    X = _f64(X, (-1, 3))
    n = X.shape[0] - 3
    H, E = np.zeros(1), np.zeros(1)
    Fg = np.zeros((n + 3, 3))
    V = np.zeros(9)
    F = np.zeros((n, 3))
    R = np.zeros((n, 3))
    h = np.zeros(9)
    _check(lib().orc_cf_eval(ctypes.byref(p), n, _d(_f64(h0, 9)), _d(X), _d(H), _d(E), _d(Fg),
                             _d(V), _d(F), _d(R), _d(h)), "cf_eval")
    return dict(H=H[0], E=E[0], Fg=Fg, V=V.reshape(3, 3), F=F, R=R, h=h.reshape(3, 3))


def build_endpoints(p, RA, hA, RB, hB):
    RA = _f64(RA, (-1, 3))
    n = RA.shape[0]
    XA = np.zeros((n + 3, 3))
    XB = np.zeros((n + 3, 3))
    _check(lib().orc_build_endpoints(ctypes.byref(p), n, _d(RA), _d(_f64(hA, 9)),
                                     _d(_f64(RB, (-1, 3))), _d(_f64(hB, 9)), _d(XA), _d(XB)),
           "build_endpoints")
    return XA, XB


def tangent_coeffs(Hm, H0, Hp):
    a = np.zeros(1)
    b = np.zeros(1)
    lib().orc_tangent_coeffs(float(Hm), float(H0), float(Hp), _d(a), _d(b))
    return a[0], b[0]


def refine_decide(X, ci, max_images, min_images, ins=(9, 4), dele=(1, 4)):
    """Decision on a band X (M x dim).  Returns (inserted_at, deleted_at, d2)."""
    X = _f64(X)
    M = X.shape[0]
    X = X.reshape(M, -1)
    ia = ctypes.c_int()
    da = ctypes.c_int()
    d2 = np.zeros(max(M - 1, 1))
    _check(lib().orc_refine_decide(M, X.shape[1], _d(X), int(ci), int(max_images), int(min_images),
                                   ins[0], ins[1], dele[0], dele[1], ctypes.byref(ia),
                                   ctypes.byref(da), _d(d2)), "refine_decide")
    return ia.value, da.value, d2[:M - 1]


def profile(X, H, Fg, natoms):
    """Path coordinate s and slopes dH/ds of a band (X, Fg: M x dim; the first natoms
    rows of 3 are atoms, taken modulo a rigid translation)."""
    X = _f64(X)
    M = X.shape[0]
    X = X.reshape(M, -1)
    Fg = _f64(Fg).reshape(M, -1)
    s = np.zeros(M)
    sl = np.zeros(M)
    _check(lib().orc_profile(M, int(natoms), X.shape[1], _d(X), _d(_f64(H, M)), _d(Fg), _d(s), _d(sl)),
           "profile")
    return s, sl


def set_threads(n):
    """Threads over which band images are evaluated (OpenMP); results do not depend on it."""
    lib().orc_set_threads(int(n))


def max_threads():
    return lib().orc_max_threads()


def path_coord(X, natoms):
    """Normalized path coordinate xi_k = s_k / s_{M-1} of a band X (M x dim; the first
    natoms rows of 3 are atoms, taken modulo a rigid translation)."""
    X = _f64(X)
    M = X.shape[0]
    X = X.reshape(M, -1)
    xi = np.zeros(M)
    _check(lib().orc_path_coord(M, int(natoms), X.shape[1], _d(X), _d(xi)), "path_coord")
    return xi


def fire_step(X, v, F, dt, alpha, n_pos, fresh, dtmax, maxstep, nmin=5, finc=1.1, fdec=0.5,
              astart=0.1, fa=0.99, roww=3):
    """One FIRE move of the band's moving images (the band step's own routine).
    X, v, F: M x dim (images 0 and M-1 fixed).  Returns (X, v, dt, alpha, n_pos, fresh)."""
    X = _f64(X).copy()
    M = X.shape[0]
    shape = X.shape
    X = X.reshape(M, -1)
    v = _f64(v).reshape(M, -1).copy()
    F = _f64(F).reshape(M, -1)
    st = FireState(float(dt), float(alpha), int(n_pos), int(fresh), 0, -1)
    _check(lib().orc_fire_step(M, X.shape[1], int(roww), _d(X), _d(v), _d(F), ctypes.byref(st),
                               float(dtmax), float(maxstep), int(nmin), float(finc), float(fdec),
                               float(astart), float(fa)), "fire_step")
    return X.reshape(shape), v.reshape(shape), st.dt, st.alpha, st.n_pos, st.fresh


def spline_eval(s, H, slope, sq):
    """Hermite interpolant through (s_k, H_k) with the given slopes, at the queries sq."""
    s = _f64(s)
    sq = _f64(sq)
    out = np.zeros(sq.size)
    _check(lib().orc_spline_eval(s.size, _d(s), _d(_f64(H)), _d(_f64(slope)), sq.size, _d(sq), _d(out)),
           "spline_eval")
    return out


def spline_max(s, H, slope):
    """(H_max, s_at) of the Hermite interpolant."""
    s = _f64(s)
    hm, at = np.zeros(1), np.zeros(1)
    _check(lib().orc_spline_max(s.size, _d(s), _d(_f64(H)), _d(_f64(slope)), _d(hm), _d(at)),
           "spline_max")
    return hm[0], at[0]


def neb2d(kappa, xy, k_spring=1.0, climb_after=0, dt0=0.01, dtmax=0.1, maxstep=0.05,
          max_steps=20000, f_tol=1e-10):
    xy = _f64(xy, (-1, 2)).copy()
    M = xy.shape[0]
    E = np.zeros(M)
    ci = ctypes.c_int()
    fmax = np.zeros(1)
    steps = lib().orc_neb2d(float(kappa), M, _d(xy), float(k_spring), int(climb_after), float(dt0),
                            float(dtmax), float(maxstep), int(max_steps), float(f_tol), _d(E),
                            ctypes.byref(ci), _d(fmax))
    return dict(xy=xy, E=E, ci=ci.value, fmax=fmax[0], steps=steps)


def relax(p, R, h, max_steps=20000, f_tol=1e-6):
    R = _f64(R, (-1, 3)).copy()
    h = _f64(h, 9).copy()
    steps = ctypes.c_int()
    fmax = np.zeros(1)
    _check(lib().orc_relax(ctypes.byref(p), R.shape[0], _d(R), _d(h), int(max_steps), float(f_tol),
                           ctypes.byref(steps), _d(fmax)), "relax")
    return R, h.reshape(3, 3), steps.value, fmax[0]


class Band:
    """The oracle's band, with the same calls as the HIP library's band."""

    def __init__(self, p, pos_init, cell_init, pos_final, cell_final, types=None):
        self.p = p
        pos_init = _f64(pos_init, (-1, 3))
        self.n = pos_init.shape[0]
        t = np.zeros(self.n, dtype=np.int32) if types is None else np.ascontiguousarray(types, np.int32)
        err = ctypes.c_int()
        self._h = lib().orc_band_create(ctypes.byref(p), self.n, _i(t), _d(pos_init),
                                        _d(_f64(cell_init, 9)), _d(_f64(pos_final, (-1, 3))),
                                        _d(_f64(cell_final, 9)), ctypes.byref(err))
        if not self._h:
            raise OracleError(err.value, "band_create")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_band_destroy(self._h)
            self._h = None

    @property
    def n_images(self):
        return lib().orc_band_n_images(self._h)

    def step(self, max_steps, f_tol=0.0):
        sd = ctypes.c_int()
        conv = ctypes.c_int()
        fmax = np.zeros(1)
        _check(lib().orc_band_step(self._h, int(max_steps), float(f_tol), ctypes.byref(sd), _d(fmax),
                                   ctypes.byref(conv)), "band_step")
        return sd.value, fmax[0], bool(conv.value)

    def refine(self):
        ia = ctypes.c_int()
        da = ctypes.c_int()
        _check(lib().orc_band_refine(self._h, ctypes.byref(ia), ctypes.byref(da)), "band_refine")
        return ia.value, da.value

    def energies(self):
        cap = self.p.max_images
        H = np.zeros(cap)
        xi = np.zeros(cap)
        M = ctypes.c_int()
        bar = np.zeros(1)
        ci = ctypes.c_int()
        _check(lib().orc_band_energies(self._h, _d(H), cap, ctypes.byref(M), _d(bar),
                                       ctypes.byref(ci), _d(xi)), "band_energies")
        return dict(H=H[:M.value].copy(), barrier=bar[0], ci=ci.value, xi=xi[:M.value].copy())

    def profile(self, n_samples=0):
        """Energy profile at the current coordinates (every image evaluated afresh)."""
        M = self.n_images
        s, H, sl = np.zeros(M), np.zeros(M), np.zeros(M)
        smp = np.zeros(max(n_samples, 1))
        bar, xm = np.zeros(1), np.zeros(1)
        _check(lib().orc_band_profile(self._h, int(n_samples), _d(s), _d(H), _d(sl), _d(smp), _d(bar),
                                      _d(xm)), "band_profile")
        return dict(s=s, H=H, slope=sl, samples=smp[:n_samples].copy(), barrier=bar[0], xi_max=xm[0])

    def get_state(self):
        cap = self.p.max_images
        dim = 3 * (self.n + 3)
        X = np.zeros((cap, self.n + 3, 3))
        v = np.zeros((cap, self.n + 3, 3))
        st = FireState()
        h0 = np.zeros(9)
        _check(lib().orc_band_get_state(self._h, _d(X), _d(v), cap, ctypes.byref(st), _d(h0)),
               "get_state")
        M = self.n_images
        del dim
        return dict(X=X[:M].copy(), v=v[:M].copy(), dt=st.dt, alpha=st.alpha, n_pos=st.n_pos,
                    fresh=st.fresh, step=st.step, ci=st.ci, h0=h0.reshape(3, 3))

    def set_state(self, X, v, dt, alpha, n_pos, fresh, step, ci=-1):
        X = _f64(X)
        M = X.shape[0]
        st = FireState(float(dt), float(alpha), int(n_pos), int(fresh), int(step), int(ci))
        _check(lib().orc_band_set_state(self._h, M, _d(X), _d(_f64(v)), ctypes.byref(st)),
               "set_state")

    def image(self, k):
        n = self.n
        E, H = np.zeros(1), np.zeros(1)
        V = np.zeros(9)
        F = np.zeros((n, 3))
        Fg = np.zeros((n + 3, 3))
        Fn = np.zeros((n + 3, 3))
        R = np.zeros((n, 3))
        h = np.zeros(9)
        _check(lib().orc_band_image(self._h, int(k), _d(E), _d(H), _d(V), _d(F), _d(Fg), _d(Fn),
                                    _d(R), _d(h)), "band_image")
        return dict(E=E[0], H=H[0], V=V.reshape(3, 3), F=F, Fg=Fg, Fneb=Fn, R=R, h=h.reshape(3, 3))
