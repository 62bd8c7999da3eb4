"""Continuous-batching request loop for f-and-gradient evaluations.

Requests (beta, D, chi, A) arrive over time.  The loop

* admits an arrived request when a slot is free and its estimated device
  footprint fits the HBM budget next to the requests already running
  (footprints per (D, chi) start from a model of the largest absorption
  intermediates and are replaced by the measured arena size of the first
  context of that shape);
* keeps the converged environments of finished requests resident in a
  per-(D, chi) pool and warm-starts a later request of the same shape from
  them (``ctm_reset_tensor``) while the pool fits the budget;
* advances all admitted requests together in slices of a few moves
  (``ctm_iterate_batch``): every move of every active request runs
  concurrently on the device, requests join between slices as they arrive and
  leave as soon as they converge, and a finished request's f and gradient are
  computed right away;
* records arrival-to-result latency per request.

All compute is in the HIP library; this module schedules.  A request's result
does not depend on which other requests share the device with it (each has
its own context and streams), except through the warm start it was given.
"""
import time
from dataclasses import dataclass, field

import numpy as np

from . import ctm

GiB = 1 << 30


@dataclass
class Request:
    rid: int
    beta: float
    A: np.ndarray            # raw PEPS tensor [2][D][D][D][D], float64
    chi: int
    t_arrival: float = 0.0   # seconds after the start of the trace
    # filled by the server
    f: float = float("nan")
    g: np.ndarray = None
    iters: int = 0
    status: int = -1
    error: str = ""          # the library's message when status is an error
    warm: bool = False
    t_admit: float = float("nan")
    t_done: float = float("nan")

    @property
    def D(self):
        return int(self.A.shape[1])

    @property
    def latency(self):
        return self.t_done - self.t_arrival


def footprint_model(D, chi, d=2):
    """Bytes of device memory one context needs, modelled on its largest
    absorption intermediates (chi^2 D^4 d^3 entries, a few dozen of them live
    per network) plus the fixed buffers (per network: a 128 MiB workspace
    chunk and the 32 MiB split-K workspace)."""
    big = chi * chi * D ** 4 * d ** 3 * 8
    return int(40 * big + 2 * 160 * (1 << 20))


@dataclass
class ServerStats:
    latencies: list = field(default_factory=list)
    wall: float = 0.0
    n_done: int = 0
    warm_starts: int = 0
    max_active: int = 0
    peak_bytes: int = 0

    def summary(self):
        lat = np.array(self.latencies) if self.latencies else np.array([np.nan])
        return dict(requests=self.n_done, wall_s=self.wall,
                    evals_per_s=self.n_done / self.wall if self.wall > 0 else float("nan"),
                    p50_latency_s=float(np.percentile(lat, 50)),
                    p99_latency_s=float(np.percentile(lat, 99)),
                    mean_latency_s=float(np.mean(lat)), warm_starts=self.warm_starts,
                    max_active=self.max_active, peak_bytes=self.peak_bytes)


class Server:
    def __init__(self, hbm_budget=96 * GiB, max_slots=16, tol=1e-9, max_iter=200, slice_moves=4,
                 warm=True, precision=ctm.CTM_FP64, lib=None, device_tensors=True):
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.tol, self.max_iter = float(tol), int(max_iter)
        self.slice = int(slice_moves)
        self.warm = bool(warm)
        self.precision = int(precision)
        self.lib = lib or ctm.load_library()
        self.device_tensors = device_tensors
        self.fp = {}          # (D, chi) -> bytes (model, then measured)
        self.pool = {}        # (D, chi) -> [idle contexts]

    # ---- bookkeeping
    def _footprint(self, D, chi):
        return self.fp.get((D, chi), footprint_model(D, chi))

    def _pool_bytes(self):
        return sum(self._footprint(*k) * len(v) for k, v in self.pool.items())

    def _tensor(self, A):
        if not self.device_tensors:
            return np.ascontiguousarray(A, dtype=np.float64)
        import torch
        return torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).cuda()

    def _context(self, req):
        key = (req.D, req.chi)
        A = self._tensor(req.A)
        if self.warm and self.pool.get(key):
            c = self.pool[key].pop()
            c.reset_tensor(req.beta, A)
            req.warm = True
            return c, A
        c = ctm.SplitCTM(req.beta, A, req.chi, max_iter=self.max_iter, tol=self.tol,
                         precision=self.precision, lib=self.lib)
        return c, A

    def _evict(self, need):
        """Drop idle pooled contexts (largest first) until `need` more bytes fit."""
        while self.pool and self._used + self._pool_bytes() + need > self.budget:
            key = max((k for k, v in self.pool.items() if v), key=lambda k: self._footprint(*k), default=None)
            if key is None:
                break
            self.pool[key].pop().close()
            if not self.pool[key]:
                del self.pool[key]

    # ---- the loop
    def run(self, requests, realtime=True, on_done=None):
        """Serve `requests` (sorted by t_arrival).  realtime: arrivals follow the
        wall clock from the start; otherwise every request is there at t = 0."""
        pending = sorted(requests, key=lambda r: r.t_arrival)
        active = []           # (req, ctx, A_keepalive)
        stats = ServerStats()
        self._used = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        i_next = 0
        reserved = {}
        while i_next < len(pending) or active:
            t = now()
            # admission: arrived, a free slot, and the footprint fits the budget
            while (i_next < len(pending) and len(active) < self.max_slots
                   and (not realtime or pending[i_next].t_arrival <= t)):
                req = pending[i_next]
                need = self._footprint(req.D, req.chi)
                warm_ok = self.warm and self.pool.get((req.D, req.chi))
                if not warm_ok:
                    self._evict(need)
                    if self._used + self._pool_bytes() + need > self.budget and active:
                        break       # wait for memory to free up
                if not realtime:
                    req.t_arrival = 0.0
                c, A = self._context(req)
                req.t_admit = now()
                self._used += need
                reserved[req.rid] = need
                active.append((req, c, A))
                i_next += 1
                stats.warm_starts += int(req.warm)
            stats.max_active = max(stats.max_active, len(active))
            if not active:
                # idle until the next arrival
                time.sleep(max(0.0, min(0.01, pending[i_next].t_arrival - now())))
                continue
            res = ctm.iterate_batch([c for _, c, _ in active], -self.slice, lib=self.lib)
            keep = []
            for (req, c, A), (done, delta, conv, st) in zip(active, res):
                req.iters += done
                if st == 0 and not conv:
                    keep.append((req, c, A))
                    continue
                req.status = st
                if st not in (0, ctm.CTM_ENOCONV):
                    req.error = c._lib.ctm_last_error(c._ctx).decode()
                if st in (0, ctm.CTM_ENOCONV):
                    try:
                        req.f = c.free_energy()[0]
                        if self.device_tensors:
                            import torch
                            g = torch.empty_like(A)
                            c.grad(g)
                            req.g = g.cpu().numpy()
                        else:
                            req.g = c.grad()
                    except ctm.CtmError as e:   # e.g. a negative network value
                        req.status = e.status
                        req.error = str(e)
                        st = e.status
                req.t_done = now()
                stats.latencies.append(req.latency)
                stats.n_done += 1
                key = (req.D, req.chi)
                _, measured = c.query()
                if key not in self.fp:
                    self.fp[key] = int(measured)
                stats.peak_bytes = max(stats.peak_bytes, self._used + self._pool_bytes())
                self._used -= reserved.pop(req.rid)
                if self.warm and st == 0:
                    self.pool.setdefault(key, []).append(c)
                    self._evict(0)
                else:
                    c.close()
                if on_done:
                    on_done(req)
            active = keep
        stats.wall = now()
        return stats

    def close(self):
        for v in self.pool.values():
            for c in v:
                c.close()
        self.pool.clear()


def trace_requests(n_requests=256, mean_rate=20.0, seed=1, D_set=None, chi_set=None):
    """The serving workload: Poisson arrivals, beta ~ U[0.18, 0.26], D and chi
    drawn per request, A the product state plus 0.3 N(0, 1) noise (seed
    1000 + i)."""
    from synth_inputs import serving_peps, serving_trace
    reqs = []
    for i, r in enumerate(serving_trace(n_requests, mean_rate, seed)):
        D = r["D"] if D_set is None else D_set[i % len(D_set)]
        chi = r["chi"] if chi_set is None else chi_set[i % len(chi_set)]
        reqs.append(Request(rid=i, beta=r["beta"], A=serving_peps(D, r["seed"]), chi=chi,
                            t_arrival=r["t_arrival"]))
    return reqs


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="replay the serving trace on one GPU")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--budget-gib", type=float, default=200.0)
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--max-iter", type=int, default=200, help="moves per request at most")
    args = ap.parse_args()
    reqs = trace_requests(args.requests, args.rate)
    srv = Server(hbm_budget=args.budget_gib * GiB, max_slots=args.slots, warm=not args.no_warm,
                 max_iter=args.max_iter)
    done = [0]

    def progress(req):
        done[0] += 1
        if done[0] % 16 == 0:
            print("served %d / %d" % (done[0], len(reqs)), flush=True)

    stats = srv.run(reqs, realtime=True, on_done=progress)
    srv.close()
    out = stats.summary()
    out["failed"] = sum(1 for r in reqs if r.status not in (0, ctm.CTM_ENOCONV))
    out["not_converged"] = sum(1 for r in reqs if r.status == ctm.CTM_ENOCONV)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
