"""Continuous-batching request loop for band relaxations.

Requests (a band to relax to a force tolerance) arrive over time.  The loop
admits waiting requests in arrival order while a batch slot is free and the sum of
the admitted bands' device footprints (cfneb_band_bytes) stays within the HBM
budget; every admitted band is made inside one batch (cfneb_batch_add) and stays
on the device until it converges, fails or reaches the step cap; between batch
calls finished bands are read out (cfneb_batch_energies) and removed
(cfneb_batch_remove), and new arrivals are admitted.  All band arithmetic runs in the HIP
library; this module only schedules.
"""
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import cfneb


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    params: object            # cfneb.Params
    endpoints: dict           # pos_init, cell_init, pos_final, cell_final
    n_atoms: int
    displace: object = None   # optional initial displacement of the interior images
    bytes: int = 0
    # filled by the server
    admitted: float = -1.0
    finished: float = -1.0
    barrier: float = float("nan")
    steps: int = 0
    moving_image_steps: int = 0
    error: int = 0
    converged: bool = False
    info: dict = field(default_factory=dict)


class Server:
    """One batch, FIFO admission by slots and HBM budget, state kept on device."""

    def __init__(self, hbm_budget_bytes, max_bands=64, f_tol=0.01, steps_per_call=32,
                 max_steps=10000, clock=time.perf_counter):
        self.budget = int(hbm_budget_bytes)
        self.max_bands = int(max_bands)
        self.f_tol = float(f_tol)
        self.steps_per_call = int(steps_per_call)
        self.max_steps = int(max_steps)
        self.clock = clock
        self.batch = None
        self.in_use = 0
        self.active = {}      # slot -> (request, band)
        self.waiting = deque()
        self.done = []
        self.occupancy = []   # (time, active bands, bytes in use)
        self.memory_waits = 0  # admissions deferred because the budget was full

    def _admit(self, now):
        while self.waiting and self.waiting[0].arrival <= now and len(self.active) < self.max_bands:
            req = self.waiting[0]
            if req.bytes > self.budget:
                self.waiting.popleft()
                req.error = -2  # CFNEB_ENOMEM: can never fit
                req.finished = now
                self.done.append(req)
                continue
            if self.in_use + req.bytes > self.budget:
                self.memory_waits += 1
                break
            self.waiting.popleft()
            e = req.endpoints
            slot = -1
            try:
                # the band is made inside the batch (cfneb_batch_add) on the batch's stream
                slot = self.batch.add(req.params, e["pos_init"], e["cell_init"], e["pos_final"],
                                      e["cell_final"])
                band = self.batch.bands[slot]
                if req.displace is not None:
                    band.displace_interior(req.displace)
            except cfneb.CfnebError as err:  # the request fails alone; the others go on
                if slot >= 0:
                    self.batch.remove(slot)
                req.error = err.code
                req.finished = self.clock() - self.t0
                self.done.append(req)
                continue
            req.admitted = self.clock() - self.t0
            self.in_use += req.bytes
            self.active[slot] = (req, band)

    def _retire(self, slot, now):
        req, band = self.active.pop(slot)
        if req.error == 0:
            e = self.batch.energies(slot)
            req.barrier = e["barrier"]
            req.info = dict(ci=e["ci"], n_images=len(e["H"]), H=e["H"])
        st = band.get_state()
        req.moving_image_steps = int(st["image_steps"])
        req.finished = now
        self.batch.remove(slot)  # destroys the band; its workspace returns to the pool
        self.in_use -= req.bytes
        self.done.append(req)

    def run(self, requests):
        """Serve every request; returns the list of finished requests."""
        for r in requests:
            r.bytes = cfneb.band_bytes(r.params, r.n_atoms)
        self.waiting = deque(sorted(requests, key=lambda r: r.arrival))
        self.batch = cfneb.Batch(self.max_bands)
        self.t0 = self.clock()
        while self.waiting or self.active:
            now = self.clock() - self.t0
            self._admit(now)
            if not self.active:
                if not self.waiting:
                    break  # the last requests were rejected at admission
                # idle until the next arrival
                nxt = self.waiting[0].arrival
                while self.clock() - self.t0 < nxt:
                    time.sleep(min(0.001, max(0.0, nxt - (self.clock() - self.t0))))
                continue
            steps, conv, errs = self.batch.step(self.steps_per_call, self.f_tol)
            now = self.clock() - self.t0
            self.occupancy.append((now, len(self.active), self.in_use))
            for slot in list(self.active):
                req, band = self.active[slot]
                req.steps += int(steps[slot])
                if errs[slot] != 0:
                    req.error = int(errs[slot])
                    self._retire(slot, now)
                elif conv[slot]:
                    req.converged = True
                    self._retire(slot, now)
                elif req.steps >= self.max_steps:
                    self._retire(slot, now)
        self.batch.close()
        return self.done


def summarize(done, wall):
    """Latency percentiles from arrival to the end of each request.

    p50_s / p99_s cover every request: a request that reached the step cap or failed is
    counted at its time to that end, a lower bound of its time to a converged barrier.
    p50_converged_s / p99_converged_s cover the converged requests alone."""
    lat_all = np.array([r.finished - r.arrival for r in done])
    lat = np.array([r.finished - r.arrival for r in done if r.error == 0 and r.converged])
    work = sum(r.n_atoms * r.moving_image_steps for r in done)

    def pct(a, q):
        return float(np.percentile(a, q)) if len(a) else None

    return dict(
        requests=len(done),
        converged=sum(r.converged for r in done),
        failed=sum(r.error != 0 for r in done),
        capped=sum((not r.converged) and r.error == 0 for r in done),
        p50_s=pct(lat_all, 50),
        p99_s=pct(lat_all, 99),
        p50_converged_s=pct(lat, 50),
        p99_converged_s=pct(lat, 99),
        atom_steps_per_s=work / wall if wall > 0 else None,
        wall_s=wall,
    )
