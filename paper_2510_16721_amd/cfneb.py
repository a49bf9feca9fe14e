"""Thin ctypes binding of libcfneb.so (the C ABI in include/cfneb.h).

Argument marshalling only: every step of the band runs in the HIP kernels of the
library.  PyTorch provides the device workspace (a uint8 tensor) and the stream.
Importing this module does not touch the GPU; loading the library fails loudly
if it has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfneb.so")

CFNEB_LJ = 1
CFNEB_TERSOFF_C = 2

ERRORS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ECELL", -5: "ENEIGH",
          -6: "ENONFINITE", -7: "ECAPACITY", -8: "ERANGE"}

# exported entry points declared in include/cfneb.h
SYMBOLS = ["cfneb_params_default", "cfneb_band_bytes", "cfneb_create_band", "cfneb_step",
           "cfneb_step_profiled",
           "cfneb_refine", "cfneb_energies", "cfneb_profile", "cfneb_get_image", "cfneb_relax",
           "cfneb_relax_noalloc", "cfneb_get_state",
           "cfneb_set_state", "cfneb_image_data", "cfneb_record_neb_force", "cfneb_neighbours",
           "cfneb_destroy", "cfneb_strerror", "cfneb_last_error", "cfneb_batch_bytes",
           "cfneb_batch_create", "cfneb_batch_attach", "cfneb_batch_detach", "cfneb_batch_add",
           "cfneb_batch_remove", "cfneb_batch_band", "cfneb_batch_energies", "cfneb_batch_step",
           "cfneb_batch_destroy"]


class Params(ctypes.Structure):
    _fields_ = [
        ("potential", ctypes.c_int), ("force_fp64", ctypes.c_int),
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
        ("nbr_cap", ctypes.c_int), ("nbr_skin", ctypes.c_double),
        ("stress_GPa", ctypes.c_double * 6),
    ]


class FireState(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("alpha", ctypes.c_double), ("n_pos", ctypes.c_int),
                ("fresh", ctypes.c_int), ("step", ctypes.c_int), ("ci", ctypes.c_int),
                ("image_steps", ctypes.c_longlong)]


PHASES = ["geom", "skin", "bins", "nlist", "filter", "force0", "force1", "force2", "reduce",
          "dots", "scalars", "update", "finalize", "move", "refine"]


_LIB = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                               "python paper_2510_16721_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _LIB = L
    return _LIB


def _declare(L):
    c_int, c_double, c_void, c_int64, c_size = (ctypes.c_int, ctypes.c_double, ctypes.c_void_p,
                                                ctypes.c_int64, ctypes.c_size_t)
    L.cfneb_params_default.argtypes = [c_int, ctypes.POINTER(Params)]
    L.cfneb_band_bytes.argtypes = [ctypes.POINTER(Params), c_int64, c_int, ctypes.POINTER(c_size)]
    L.cfneb_create_band.argtypes = [ctypes.POINTER(Params), c_int64, _ip, _dp, _dp, _dp, _dp,
                                    c_void, c_size, c_void, ctypes.POINTER(c_void)]
    L.cfneb_step.argtypes = [c_void, c_int, c_double, ctypes.POINTER(c_int), _dp,
                             ctypes.POINTER(c_int)]
    L.cfneb_step_profiled.argtypes = [c_void, c_int, c_double, ctypes.POINTER(c_int), _dp,
                                      ctypes.POINTER(c_int), _dp, c_int]
    L.cfneb_refine.argtypes = [c_void, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    L.cfneb_energies.argtypes = [c_void, _dp, c_int, ctypes.POINTER(c_int), _dp,
                                 ctypes.POINTER(c_int), _dp]
    L.cfneb_profile.argtypes = [c_void, c_int, _dp, _dp, _dp, c_int, ctypes.POINTER(c_int), _dp, _dp,
                                _dp]
    L.cfneb_get_image.argtypes = [c_void, c_int, _dp, _dp]
    L.cfneb_relax.argtypes = [ctypes.POINTER(Params), c_int64, _ip, _dp, _dp, c_int, c_double,
                              c_void, c_size, c_void, ctypes.POINTER(c_int), _dp,
                              ctypes.POINTER(c_int)]
    L.cfneb_relax_noalloc.argtypes = [ctypes.POINTER(Params), c_int64, _ip, _dp, _dp, c_int, c_double,
                                      c_void, ctypes.POINTER(c_int), _dp, ctypes.POINTER(c_int)]
    L.cfneb_get_state.argtypes = [c_void, _dp, _dp, c_int, ctypes.POINTER(c_int),
                                  ctypes.POINTER(FireState)]
    L.cfneb_set_state.argtypes = [c_void, c_int, _dp, _dp, ctypes.POINTER(FireState)]
    L.cfneb_image_data.argtypes = [c_void, c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.cfneb_record_neb_force.argtypes = [c_void, c_int]
    L.cfneb_neighbours.argtypes = [c_void, c_int, _ip, _ip, c_int64, ctypes.POINTER(c_int64)]
    L.cfneb_destroy.argtypes = [c_void]
    L.cfneb_strerror.argtypes = [c_int]
    L.cfneb_strerror.restype = ctypes.c_char_p
    L.cfneb_last_error.argtypes = [c_void]
    L.cfneb_last_error.restype = ctypes.c_char_p
    L.cfneb_batch_bytes.argtypes = [c_int, ctypes.POINTER(c_size)]
    L.cfneb_batch_create.argtypes = [c_int, c_void, c_size, c_void, ctypes.POINTER(c_void)]
    L.cfneb_batch_attach.argtypes = [c_void, c_void, ctypes.POINTER(c_int)]
    L.cfneb_batch_detach.argtypes = [c_void, c_int]
    L.cfneb_batch_add.argtypes = [c_void, ctypes.POINTER(Params), c_int64, _ip, _dp, _dp, _dp, _dp,
                                  c_void, c_size, ctypes.POINTER(c_int)]
    L.cfneb_batch_remove.argtypes = [c_void, c_int]
    L.cfneb_batch_band.argtypes = [c_void, c_int]
    L.cfneb_batch_band.restype = c_void
    L.cfneb_batch_energies.argtypes = [c_void, c_int, _dp, c_int, ctypes.POINTER(c_int), _dp,
                                       ctypes.POINTER(c_int), _dp]
    L.cfneb_batch_step.argtypes = [c_void, c_int, c_double, _ip, ctypes.POINTER(ctypes.c_uint8), _ip]
    L.cfneb_batch_destroy.argtypes = [c_void]


class CfnebError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def default_params(potential, **kw):
    p = Params()
    rc = lib().cfneb_params_default(int(potential), ctypes.byref(p))
    if rc != 0:
        raise CfnebError(rc, "cfneb_params_default")
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    if "fire_dt0" in kw and "fire_dtmax" not in kw:
        p.fire_dtmax = 10.0 * p.fire_dt0
    return p


def band_bytes(p, n_atoms, max_images=0):
    out = ctypes.c_size_t()
    rc = lib().cfneb_band_bytes(ctypes.byref(p), int(n_atoms), int(max_images), ctypes.byref(out))
    if rc != 0:
        raise CfnebError(rc, "cfneb_band_bytes")
    return out.value


def relax(p, pos, cell, max_steps=20000, f_tol=1e-4, stream=None):
    """Cell-filter relaxation of one structure on the current HIP device.
    Returns (pos, cell, steps, fmax, converged); the inputs are not modified."""
    import torch
    R = _f64(pos, (-1, 3)).copy()
    h = _f64(cell, 9).copy()
    nbytes = band_bytes(p, R.shape[0], 3)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = ws.data_ptr()
    ptr = (base + 255) // 256 * 256
    stream = stream if stream is not None else torch.cuda.current_stream()
    steps, conv = ctypes.c_int(), ctypes.c_int()
    fmax = np.zeros(1)
    rc = lib().cfneb_relax(ctypes.byref(p), R.shape[0], None, _d(R), _d(h), int(max_steps),
                           float(f_tol), ctypes.c_void_p(ptr), ws.numel() - (ptr - base),
                           ctypes.c_void_p(stream.cuda_stream), ctypes.byref(steps), _d(fmax),
                           ctypes.byref(conv))
    if rc != 0:
        raise CfnebError(rc, "cfneb_relax")
    return R, h.reshape(3, 3), steps.value, fmax[0], bool(conv.value)


# device bytes of the static array behind cfneb_relax_noalloc
RELAX_SCRATCH_BYTES = 64 << 20


def relax_noalloc(p, pos, cell, max_steps=20000, f_tol=1e-4, stream=None):
    """cfneb_relax_noalloc: the relaxation of relax() with the library's static device
    array instead of a workspace (nothing is allocated).  Same return value."""
    import torch
    R = _f64(pos, (-1, 3)).copy()
    h = _f64(cell, 9).copy()
    stream = stream if stream is not None else torch.cuda.current_stream()
    steps, conv = ctypes.c_int(), ctypes.c_int()
    fmax = np.zeros(1)
    rc = lib().cfneb_relax_noalloc(ctypes.byref(p), R.shape[0], None, _d(R), _d(h), int(max_steps),
                                   float(f_tol), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(steps),
                                   _d(fmax), ctypes.byref(conv))
    if rc != 0:
        raise CfnebError(rc, "cfneb_relax_noalloc")
    return R, h.reshape(3, 3), steps.value, fmax[0], bool(conv.value)


class Band:
    """One band on the current HIP device.  The workspace is a torch uint8 tensor."""

    def __init__(self, p, pos_init, cell_init, pos_final, cell_final, stream=None, workspace=None):
        import torch
        self.p = p
        pos_init = _f64(pos_init, (-1, 3))
        self.n = pos_init.shape[0]
        nbytes = band_bytes(p, self.n)
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self._ws = workspace
        base = workspace.data_ptr()
        self._ptr = (base + 255) // 256 * 256
        self._ws_bytes = workspace.numel() - (self._ptr - base)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = lib().cfneb_create_band(ctypes.byref(p), self.n, None, _d(pos_init),
                                     _d(_f64(cell_init, 9)), _d(_f64(pos_final, (-1, 3))),
                                     _d(_f64(cell_final, 9)), ctypes.c_void_p(self._ptr),
                                     self._ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h))
        if rc != 0:
            raise CfnebError(rc, "cfneb_create_band")
        self._h = h

    def _check(self, rc, what):
        if rc != 0:
            msg = lib().cfneb_last_error(self._h).decode()
            raise CfnebError(rc, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            lib().cfneb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def bytes(self):
        return self._ws_bytes

    def step(self, max_steps, f_tol=0.0):
        sd = ctypes.c_int()
        conv = ctypes.c_int()
        fmax = ctypes.c_double()
        rc = lib().cfneb_step(self._h, int(max_steps), float(f_tol), ctypes.byref(sd),
                              ctypes.byref(fmax), ctypes.byref(conv))
        self._check(rc, "cfneb_step")
        return sd.value, fmax.value, bool(conv.value)

    def step_profiled(self, max_steps, f_tol=0.0):
        """Steps with per-phase HIP-event timing; returns (steps, fmax, converged, {phase: ms})."""
        sd = ctypes.c_int()
        conv = ctypes.c_int()
        fmax = ctypes.c_double()
        ms = np.zeros(len(PHASES))
        rc = lib().cfneb_step_profiled(self._h, int(max_steps), float(f_tol), ctypes.byref(sd),
                                       ctypes.byref(fmax), ctypes.byref(conv), _d(ms), len(PHASES))
        self._check(rc, "cfneb_step_profiled")
        return sd.value, fmax.value, bool(conv.value), dict(zip(PHASES, ms.tolist()))

    def refine(self):
        ia = ctypes.c_int()
        da = ctypes.c_int()
        self._check(lib().cfneb_refine(self._h, ctypes.byref(ia), ctypes.byref(da)), "cfneb_refine")
        return ia.value, da.value

    def energies(self):
        cap = 64
        H = np.zeros(cap)
        xi = np.zeros(cap)
        M = ctypes.c_int()
        bar = ctypes.c_double()
        ci = ctypes.c_int()
        self._check(lib().cfneb_energies(self._h, _d(H), cap, ctypes.byref(M), ctypes.byref(bar),
                                         ctypes.byref(ci), _d(xi)), "cfneb_energies")
        return dict(H=H[:M.value].copy(), barrier=bar.value, ci=ci.value, xi=xi[:M.value].copy())

    def profile(self, n_samples=0):
        """Energy profile at the current coordinates (every image evaluated afresh):
        arc length s, H and slope dH/ds per image, n_samples evenly spaced samples of
        the Hermite interpolant over the normalized coordinate, its maximum minus H_0
        and where that maximum lies."""
        cap = 64
        s, H, sl = np.zeros(cap), np.zeros(cap), np.zeros(cap)
        smp = np.zeros(max(int(n_samples), 1))
        M = ctypes.c_int()
        bar, xm = ctypes.c_double(), ctypes.c_double()
        self._check(lib().cfneb_profile(self._h, int(n_samples), _d(s), _d(H), _d(sl), cap, ctypes.byref(M),
                                        _d(smp), ctypes.byref(bar), ctypes.byref(xm)), "cfneb_profile")
        m = M.value
        return dict(s=s[:m].copy(), H=H[:m].copy(), slope=sl[:m].copy(), samples=smp[:n_samples].copy(),
                    barrier=bar.value, xi_max=xm.value)

    def get_image(self, k):
        pos = np.zeros((self.n, 3))
        cell = np.zeros(9)
        self._check(lib().cfneb_get_image(self._h, int(k), _d(pos), _d(cell)), "cfneb_get_image")
        return pos, cell.reshape(3, 3)

    def get_state(self):
        cap = 64
        rows = self.n + 3
        M = ctypes.c_int()
        st = FireState()
        self._check(lib().cfneb_get_state(self._h, None, None, 0, ctypes.byref(M), ctypes.byref(st)),
                    "cfneb_get_state")
        X = np.zeros((M.value, rows, 3))
        v = np.zeros((M.value, rows, 3))
        self._check(lib().cfneb_get_state(self._h, _d(X), _d(v), M.value, ctypes.byref(M),
                                          ctypes.byref(st)), "cfneb_get_state")
        del cap
        return dict(X=X, v=v, dt=st.dt, alpha=st.alpha, n_pos=st.n_pos, fresh=st.fresh,
                    step=st.step, ci=st.ci, image_steps=st.image_steps)

    def set_state(self, X, v, dt, alpha, n_pos, fresh, step, ci=-1):
        X = _f64(X)
        st = FireState(float(dt), float(alpha), int(n_pos), int(fresh), int(step), int(ci), 0)
        vv = _f64(v) if v is not None else None
        self._check(lib().cfneb_set_state(self._h, X.shape[0], _d(X),
                                          _d(vv) if vv is not None else None, ctypes.byref(st)),
                    "cfneb_set_state")

    def displace_interior(self, d):
        """Add d (n_images - 2, n_atoms, 3) to the atom rows R~ of the interior images."""
        st = self.get_state()
        X = st["X"]
        d = _f64(d, (X.shape[0] - 2, self.n, 3))
        X[1:-1, :self.n] += d
        self.set_state(X, st["v"], st["dt"], st["alpha"], st["n_pos"], st["fresh"], st["step"],
                       st["ci"])

    def record_neb_force(self, on=True):
        self._check(lib().cfneb_record_neb_force(self._h, 1 if on else 0), "cfneb_record_neb_force")

    def image(self, k):
        n = self.n
        E, H = ctypes.c_double(), ctypes.c_double()
        V = np.zeros(9)
        F = np.zeros((n, 3))
        Fg = np.zeros((n + 3, 3))
        Fn = np.zeros((n + 3, 3))
        R = np.zeros((n, 3))
        h = np.zeros(9)
        self._check(lib().cfneb_image_data(self._h, int(k), ctypes.byref(E), ctypes.byref(H), _d(V),
                                           _d(F), _d(Fg), _d(Fn), _d(R), _d(h)), "cfneb_image_data")
        return dict(E=E.value, H=H.value, V=V.reshape(3, 3), F=F, Fg=Fg, Fneb=Fn, R=R,
                    h=h.reshape(3, 3))

    def neighbours(self, k):
        n = self.n
        cnt = np.zeros(n, dtype=np.int32)
        tot = ctypes.c_int64()
        self._check(lib().cfneb_neighbours(self._h, int(k), cnt.ctypes.data_as(_ip), None, 0,
                                           ctypes.byref(tot)), "cfneb_neighbours")
        ent = np.zeros((max(tot.value, 1), 4), dtype=np.int32)
        self._check(lib().cfneb_neighbours(self._h, int(k), cnt.ctypes.data_as(_ip),
                                           ent.ctypes.data_as(_ip), ent.shape[0], ctypes.byref(tot)),
                    "cfneb_neighbours")
        cap = self.p.nbr_cap
        off = np.concatenate([[0], np.cumsum(np.minimum(cnt, cap))])
        return cnt, [ent[off[i]:off[i + 1]].copy() for i in range(n)]


class _OwnedBand(Band):
    """Per-band calls on a band that a batch made (cfneb_batch_add): the batch destroys it."""

    def __init__(self, handle, p, n, workspace, stream):
        self.p = p
        self.n = n
        self._ws = workspace
        self._ws_bytes = workspace.numel()
        self.stream = stream
        self._h = ctypes.c_void_p(handle)

    def close(self):
        self._h = None  # owned by the batch


def batch_bytes(max_bands):
    out = ctypes.c_size_t()
    rc = lib().cfneb_batch_bytes(int(max_bands), ctypes.byref(out))
    if rc != 0:
        raise CfnebError(rc, "cfneb_batch_bytes")
    return out.value


class Batch:
    """Many bands stepped together: one persistent launch per phase over all of them."""

    def __init__(self, max_bands, stream=None):
        import torch
        self.cap = int(max_bands)
        nbytes = batch_bytes(self.cap)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = lib().cfneb_batch_create(self.cap, ctypes.c_void_p(ptr), self._ws.numel() - (ptr - base),
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise CfnebError(rc, "cfneb_batch_create")
        self._h = h
        self.bands = [None] * self.cap

    def attach(self, band):
        slot = ctypes.c_int()
        rc = lib().cfneb_batch_attach(self._h, band._h, ctypes.byref(slot))
        if rc != 0:
            raise CfnebError(rc, "cfneb_batch_attach")
        self.bands[slot.value] = band
        return slot.value

    def detach(self, slot):
        rc = lib().cfneb_batch_detach(self._h, int(slot))
        if rc != 0:
            raise CfnebError(rc, "cfneb_batch_detach")
        self.bands[slot] = None

    def add(self, p, pos_init, cell_init, pos_final, cell_final, workspace=None):
        """Create a band owned by the batch (cfneb_batch_add); returns its slot.  The
        workspace tensor is kept alive until the band is removed."""
        import torch
        pos_init = _f64(pos_init, (-1, 3))
        n = pos_init.shape[0]
        if workspace is None:
            workspace = torch.empty(band_bytes(p, n) + 256, dtype=torch.uint8, device="cuda")
        base = workspace.data_ptr()
        ptr = (base + 255) // 256 * 256
        slot = ctypes.c_int()
        rc = lib().cfneb_batch_add(self._h, ctypes.byref(p), n, None, _d(pos_init), _d(_f64(cell_init, 9)),
                                   _d(_f64(pos_final, (-1, 3))), _d(_f64(cell_final, 9)),
                                   ctypes.c_void_p(ptr), workspace.numel() - (ptr - base),
                                   ctypes.byref(slot))
        if rc != 0:
            raise CfnebError(rc, "cfneb_batch_add")
        self.bands[slot.value] = _OwnedBand(lib().cfneb_batch_band(self._h, slot.value), p, n, workspace,
                                            self.stream)
        return slot.value

    def remove(self, slot):
        """Detach the band in `slot`; a band made by add() is destroyed."""
        rc = lib().cfneb_batch_remove(self._h, int(slot))
        if rc != 0:
            raise CfnebError(rc, "cfneb_batch_remove")
        b = self.bands[slot]
        if isinstance(b, _OwnedBand):
            b._h = None  # destroyed by the library
        self.bands[slot] = None

    def energies(self, slot):
        """cfneb_batch_energies: H, barrier, climbing image and path coordinate of a slot."""
        cap = 64
        H = np.zeros(cap)
        xi = np.zeros(cap)
        M = ctypes.c_int()
        bar = ctypes.c_double()
        ci = ctypes.c_int()
        rc = lib().cfneb_batch_energies(self._h, int(slot), _d(H), cap, ctypes.byref(M), ctypes.byref(bar),
                                        ctypes.byref(ci), _d(xi))
        if rc != 0:
            raise CfnebError(rc, "cfneb_batch_energies")
        return dict(H=H[:M.value].copy(), barrier=bar.value, ci=ci.value, xi=xi[:M.value].copy())

    def step(self, max_steps, f_tol=0.0):
        """Returns (steps per slot, converged per slot, error code per slot)."""
        steps = np.zeros(self.cap, dtype=np.int32)
        conv = np.zeros(self.cap, dtype=np.uint8)
        errs = np.zeros(self.cap, dtype=np.int32)
        rc = lib().cfneb_batch_step(self._h, int(max_steps), float(f_tol), steps.ctypes.data_as(_ip),
                                    conv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                    errs.ctypes.data_as(_ip))
        if rc != 0:
            raise CfnebError(rc, "cfneb_batch_step")
        return steps, conv.astype(bool), errs

    def close(self):
        if getattr(self, "_h", None):
            lib().cfneb_batch_destroy(self._h)
            self._h = None
            for b in self.bands:
                if isinstance(b, _OwnedBand):
                    b._h = None  # destroyed with the batch

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
