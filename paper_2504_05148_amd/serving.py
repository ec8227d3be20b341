"""Continuous-batching serving loop over the sldf C ABI.

Several rigs (camera pair + LiDAR, each with its own resolution and
disparity range) send frames as they are captured.  Per-rig state stays on
the device: every rig owns a set of slots, a slot being one context with its
workspace, pinned host staging and device input / output buffers for up to
`max_batch` frames.  Slots are created lazily while the HBM budget allows
(the slot's bytes = the library's exact workspace size plus its buffers), so
admission is by HBM budget.  The scheduler

  - moves arrived requests into per-rig queues,
  - retires finished launches (event polling; no host-wide synchronisation),
  - admits queued requests whenever a slot of their rig and a stream are
    free: all requests of that rig waiting at that moment (up to max_batch)
    go into one batched call, so requests that arrive while others are on
    the GPU join the next launch, and launches of different rigs overlap on
    different streams,

and records latency = completion - arrival for every request.

Failure handling, per rig (the other rigs are never affected):
  - a rig whose parameters the library rejects (the backend's slot size
    raises, e.g. an invalid shape or a 16-bit overflow bound) or whose one
    slot is larger than the whole HBM budget is rejected at admission: its
    requests fail at once instead of waiting for a slot that cannot exist;
  - a failed launch fails its requests and returns its slot and stream;
  - when the budget is full and a rig with waiting requests owns no slot, an
    idle slot of another rig is released to make room;
  - a rig that has sent nothing for `idle_timeout` seconds and has nothing
    in flight gets its slots (its device state) released.

The backend is an interface so the scheduler runs on the CPU in tests
(`FakeBackend`); `SldfBackend` runs the library on the GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import os
import sys
import time
from typing import Any

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    rig: int
    frame: int
    arrival: float          # seconds since the start of the run
    start: float = -1.0
    done: float = -1.0
    batch: int = 0


class FakeBackend:
    """CPU stand-in: a launch takes `cost[rig] * n_frames` seconds after it is
    enqueued on an idle stream; streams run in parallel.  Slots cost
    `slot_bytes[rig]` of budget.  Optional failure injection: launches of the
    rigs in `fail_rigs` raise."""

    def __init__(self, cost, slot_bytes, fail_rigs=(), bad_rigs=()):
        self.cost = cost
        self.slot_bytes_ = slot_bytes
        self.fail_rigs = set(fail_rigs)
        self.bad_rigs = set(bad_rigs)       # parameters the library would reject
        self.clock = time.perf_counter
        self.live = 0                       # slots made and not yet freed
        self.freed = []

    def slot_bytes(self, rig):
        if rig in self.bad_rigs:
            raise ValueError(f"rig {rig}: invalid parameters")
        return self.slot_bytes_[rig]

    def make_slot(self, rig):
        self.live += 1
        return dict(rig=rig)

    def free_slot(self, slot):
        self.live -= 1
        self.freed.append(slot["rig"])

    def enqueue(self, slot, stream, reqs):
        if slot["rig"] in self.fail_rigs:
            raise RuntimeError("injected device failure")
        return dict(t_done=self.clock() + self.cost[slot["rig"]] * len(reqs))

    def done(self, handle):
        return self.clock() >= handle["t_done"]

    def n_streams(self):
        return 4


class Server:
    def __init__(self, backend, n_rigs, hbm_budget, max_batch=4, n_streams=None,
                 idle_timeout=None):
        self.be = backend
        self.n_rigs = n_rigs
        self.budget = hbm_budget
        self.max_batch = max_batch
        self.idle_timeout = idle_timeout
        self.streams = list(range(n_streams or backend.n_streams()))
        self.slots = {r: [] for r in range(n_rigs)}      # all slots of a rig
        self.free = {r: [] for r in range(n_rigs)}       # idle slots
        self.used_bytes = 0
        self.peak_bytes = 0
        self.failed: list[Request] = []
        self.rejected: dict[int, str] = {}               # rig -> reason
        self._bytes: dict[int, int] = {}                 # rig -> bytes of one slot
        self.released = collections.Counter()            # rig -> slots released
        self.batches = collections.Counter()

    def _slot_bytes(self, rig):
        """Bytes of one slot of the rig, or None when the rig is rejected
        (parameters the library refuses, or a slot larger than the budget)."""
        if rig in self.rejected:
            return None
        if rig not in self._bytes:
            try:
                b = int(self.be.slot_bytes(rig))
            except Exception as e:      # invalid parameters: reject this rig only
                self.rejected[rig] = f"parameters rejected: {e}"
                return None
            if b > self.budget:
                self.rejected[rig] = (f"one slot ({b} B) exceeds the HBM budget "
                                      f"({self.budget} B)")
                return None
            self._bytes[rig] = b
        return self._bytes[rig]

    def _new_slot(self, rig, b):
        slot = self.be.make_slot(rig)
        self.used_bytes += b
        self.peak_bytes = max(self.peak_bytes, self.used_bytes)
        self.slots[rig].append(slot)
        return slot

    def _release(self, rig, slot):
        """Release an idle slot (its context and buffers) of a rig."""
        self.free[rig].remove(slot)
        self.slots[rig].remove(slot)
        self.used_bytes -= self._bytes[rig]
        self.be.free_slot(slot)
        self.released[rig] += 1

    def preallocate(self, per_rig):
        """Create up to per_rig idle slots per rig (round-robin, within the
        budget) so that no allocation happens while serving."""
        for _ in range(per_rig):
            for rig in range(self.n_rigs):
                b = self._slot_bytes(rig)
                if b is None or self.used_bytes + b > self.budget:
                    continue
                self.free[rig].append(self._new_slot(rig, b))

    def _get_slot(self, rig):
        """An idle slot of the rig, a new one within the budget (releasing
        idle slots of other rigs when the budget is full and the rig owns
        none), or None (wait for one of its slots, or the rig is rejected)."""
        if self.free[rig]:
            return self.free[rig].pop()
        b = self._slot_bytes(rig)
        if b is None:
            return None
        if self.used_bytes + b > self.budget and not self.slots[rig]:
            # the rig owns no slot at all: take room from idle slots of the
            # rigs holding the most of them
            while self.used_bytes + b > self.budget:
                donors = [r for r in range(self.n_rigs) if r != rig and self.free[r]]
                if not donors:
                    break
                d = max(donors, key=lambda r: len(self.free[r]))
                self._release(d, self.free[d][0])
        if self.used_bytes + b > self.budget:
            return None
        return self._new_slot(rig, b)

    def run(self, arrivals, realtime=True, progress=None):
        """arrivals: list of (t, rig, frame) sorted by t.  Returns the list of
        finished Requests (failed ones in self.failed)."""
        reqs = [Request(i, r, f, t) for i, (t, r, f) in enumerate(arrivals)]
        pending = collections.deque(reqs)
        queues = {r: collections.deque() for r in range(self.n_rigs)}
        in_flight = []          # (handle, slot, stream, [requests])
        free_streams = list(self.streams)
        finished = []
        clock = self.be.clock
        t0 = clock()
        last_report = t0
        last_seen = {r: 0.0 for r in range(self.n_rigs)}     # last arrival per rig
        while pending or in_flight or any(queues.values()):
            now = clock() - t0
            if not realtime and not in_flight and not any(queues.values()) and pending:
                t0 -= pending[0].arrival - now      # skip idle time in simulations
                now = clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                last_seen[r.rig] = r.arrival
                if self._slot_bytes(r.rig) is None:
                    self.failed.append(r)         # rejected rig: fail at admission
                else:
                    queues[r.rig].append(r)
            # rigs silent for longer than the timeout release their idle slots
            if self.idle_timeout is not None:
                for rig in range(self.n_rigs):
                    if (self.free[rig] and not queues[rig]
                            and len(self.free[rig]) == len(self.slots[rig])
                            and now - last_seen[rig] > self.idle_timeout):
                        for slot in list(self.free[rig]):
                            self._release(rig, slot)
            # retire finished launches
            still = []
            for h, slot, st, batch in in_flight:
                if self.be.done(h):
                    tdone = clock() - t0
                    for r in batch:
                        r.done = tdone
                        finished.append(r)
                    self.free[slot_rig(slot, batch)].append(slot)
                    free_streams.append(st)
                else:
                    still.append((h, slot, st, batch))
            in_flight = still
            # admit: oldest waiting request first, whole rig queue per launch
            while free_streams:
                heads = [(q[0].arrival, rig) for rig, q in queues.items() if q]
                if not heads:
                    break
                admitted = False
                for _, rig in sorted(heads):
                    slot = self._get_slot(rig)
                    if slot is None:
                        continue
                    q = queues[rig]
                    batch = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
                    st = free_streams.pop()
                    tstart = clock() - t0
                    for r in batch:
                        r.start = tstart
                        r.batch = len(batch)
                    try:
                        h = self.be.enqueue(slot, st, batch)
                    except Exception:
                        # the launch failed: its requests fail, slot and stream
                        # go back, the loop continues with the other rigs
                        self.failed.extend(batch)
                        self.free[rig].append(slot)
                        free_streams.append(st)
                        admitted = True
                        break
                    self.batches[len(batch)] += 1
                    in_flight.append((h, slot, st, batch))
                    admitted = True
                    break
                if not admitted:
                    break
            if progress and clock() - last_report > 1.0:
                last_report = clock()
                progress(len(finished), len(reqs))
            if realtime:
                time.sleep(5e-5)
        return finished


def slot_rig(slot, batch):
    return batch[0].rig


def poisson_arrivals(rates, duration, pool_size, seed=5):
    """Exponential inter-arrival times per rig from default_rng([seed, rig]);
    frames drawn round-robin from the rig's pool."""
    out = []
    for rig, rate in enumerate(rates):
        rng = np.random.default_rng([seed, rig])
        t, k = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= duration:
                break
            out.append((t, rig, k % pool_size))
            k += 1
    out.sort()
    return out


def summarize(finished, failed, duration_wall, n_rigs):
    lat = np.array([r.done - r.arrival for r in finished]) * 1e3
    per = {}
    for rig in range(n_rigs):
        lr = np.array([r.done - r.arrival for r in finished if r.rig == rig]) * 1e3
        if lr.size:
            per[rig] = dict(n=int(lr.size), p50_ms=round(float(np.percentile(lr, 50)), 3),
                            p99_ms=round(float(np.percentile(lr, 99)), 3))
    return dict(requests=len(finished) + len(failed), completed=len(finished),
                failed=len(failed), frames_per_s=round(len(finished) / duration_wall, 2),
                p50_ms=round(float(np.percentile(lat, 50)), 3) if lat.size else None,
                p99_ms=round(float(np.percentile(lat, 99)), 3) if lat.size else None,
                per_rig=per)


# --------------------------------------------------------------- GPU backend --
class SldfBackend:
    """One slot = one sldf context (batch = max_batch) with pinned host
    staging and device buffers; a launch = H2D copies + LiDAR ingest +
    sldf_run_batch on the slot's stream, completion by a recorded event."""

    def __init__(self, rigs, pools, max_batch, check_impl=0, surrogate=None, n_streams=8,
                 keep_outputs=False):
        import torch
        from paper_2504_05148_amd import sldf
        self.torch, self.sldf = torch, sldf
        self.rigs = rigs                    # list of dicts W, H, D
        self.pools = pools                  # rig -> dict of pinned host arrays
        self.max_batch = max_batch
        self.check_impl = check_impl
        self.surrogate = surrogate
        # default priority streams only
        self._streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.keep_outputs = keep_outputs
        self.outputs = {}                   # (rig, frame) -> list of (disp, valid) host copies
        self.clock = time.perf_counter

    def n_streams(self):
        return len(self._streams)

    def _params(self, rig):
        r = self.rigs[rig]
        return self.sldf.default_params(width=r["W"], height=r["H"], max_disp=r["D"],
                                        batch=self.max_batch, check_impl=self.check_impl)

    def slot_bytes(self, rig):
        r = self.rigs[rig]
        B, H, W = self.max_batch, r["H"], r["W"]
        pitch = (W + 15) // 16 * 16
        buffers = B * H * (2 * pitch + 4 * W + 2 * W + 4 * W + W)
        return self.sldf.workspace_size(self._params(rig)) + buffers

    def make_slot(self, rig):
        torch = self.torch
        r = self.rigs[rig]
        B, H, W = self.max_batch, r["H"], r["W"]
        pitch = (W + 15) // 16 * 16
        ctx = self.sldf.Context(self._params(rig))
        if self.check_impl:
            ctx.set_surrogate(*self.surrogate)
        dev = "cuda"
        slot = dict(rig=rig, ctx=ctx,
                    left=torch.zeros((B, H, pitch), dtype=torch.uint8, device=dev),
                    right=torch.zeros((B, H, pitch), dtype=torch.uint8, device=dev),
                    lid=torch.empty((B, H, W), dtype=torch.float32, device=dev),
                    lq=torch.empty((B, H, W), dtype=torch.int16, device=dev),
                    disp=torch.empty((B, H, W), dtype=torch.float32, device=dev),
                    valid=torch.empty((B, H, W), dtype=torch.uint8, device=dev),
                    event=torch.cuda.Event())
        # the zero fills above run on the creating (default) stream, which is
        # not ordered with the launch streams: finish them before first use
        torch.cuda.current_stream().synchronize()
        return slot

    def free_slot(self, slot):
        slot["ctx"].close()

    def enqueue(self, slot, stream_idx, reqs):
        torch = self.torch
        st = self._streams[stream_idx]
        pool = self.pools[slot["rig"]]
        n = len(reqs)
        r = self.rigs[slot["rig"]]
        W, D = r["W"], r["D"]
        with torch.cuda.stream(st):
            for i, q in enumerate(reqs):
                slot["left"][i, :, :W].copy_(pool["left"][q.frame], non_blocking=True)
                slot["right"][i, :, :W].copy_(pool["right"][q.frame], non_blocking=True)
                slot["lid"][i].copy_(pool["lidar"][q.frame], non_blocking=True)
            H = r["H"]
            self.sldf.quantize_lidar(slot["lid"][:n].reshape(n * H, W), D,
                                     out=slot["lq"][:n].reshape(n * H, W), stream=st)
            slot["ctx"].run_batch(slot["left"][:n, :, :W], slot["right"][:n, :, :W],
                                  slot["lq"][:n], slot["disp"][:n], slot["valid"][:n], stream=st)
            if self.keep_outputs:
                for i, q in enumerate(reqs):
                    key = (q.rig, q.frame)
                    self.outputs.setdefault(key, []).append(
                        (slot["disp"][i].to("cpu", non_blocking=True),
                         slot["valid"][i].to("cpu", non_blocking=True)))
            slot["event"].record(st)
        return slot["event"]

    def done(self, event):
        return event.query()


def _gen(args):
    rig, idx = args
    from paper_2504_05148_amd import synth
    f = synth.make_frame(synth.serving_spec(rig), synth.CONFIG_IDS["serving"], rig * 1000 + idx)
    return rig, idx, f["left"], f["right"], f["lidar"]


def make_pools(n_rigs, pool_size, workers=14):
    """Seeded frame pools per rig in pinned host memory."""
    import torch
    from multiprocessing import Pool
    from paper_2504_05148_amd import synth
    pools = {}
    for rig in range(n_rigs):
        s = synth.serving_spec(rig)
        pools[rig] = dict(
            left=torch.empty((pool_size, s.H, s.W), dtype=torch.uint8, pin_memory=True),
            right=torch.empty((pool_size, s.H, s.W), dtype=torch.uint8, pin_memory=True),
            lidar=torch.empty((pool_size, s.H, s.W), dtype=torch.float32, pin_memory=True))
    jobs = [(rig, i) for rig in range(n_rigs) for i in range(pool_size)]
    with Pool(workers) as p:
        for rig, i, L, R, lid in p.imap_unordered(_gen, jobs):
            pools[rig]["left"][i].copy_(torch.from_numpy(L))
            pools[rig]["right"][i].copy_(torch.from_numpy(R))
            pools[rig]["lidar"][i].copy_(torch.from_numpy(lid))
    return pools


def run_serving(duration=5.0, pool_size=16, max_batch=4, hbm_budget=96 << 30,
                check_impl=0, surrogate=None, pools=None, rates=None, keep_outputs=False,
                n_streams=8, log=None, prealloc=3, idle_timeout=1.0):
    """Run the six-rig mix on the GPU; returns (summary dict, backend, finished).
    Rigs that send nothing for idle_timeout seconds release their slots."""
    import torch
    from paper_2504_05148_amd import synth
    n_rigs = len(synth.SERVING_RIGS)
    rigs = [dict(W=r["W"], H=r["H"], D=r["D"]) for r in synth.SERVING_RIGS]
    if pools is None:
        pools = make_pools(n_rigs, pool_size)
    rates = rates or [50.0] * n_rigs
    be = SldfBackend(rigs, pools, max_batch, check_impl, surrogate, n_streams=n_streams,
                     keep_outputs=keep_outputs)
    srv = Server(be, n_rigs, hbm_budget, max_batch, idle_timeout=idle_timeout)
    srv.preallocate(prealloc)
    # warm-up: one launch per rig
    warm = [(0.0, rig, 0) for rig in range(n_rigs)]
    srv.run(warm, realtime=False)
    torch.cuda.synchronize()
    be.outputs.clear()
    arr = poisson_arrivals(rates, duration, pool_size)
    t0 = time.perf_counter()
    fin = srv.run(arr, progress=log)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    summ = summarize(fin, srv.failed, wall, n_rigs)
    summ.update(batches=dict(sorted(srv.batches.items())), peak_slot_bytes=srv.peak_bytes,
                budget_bytes=hbm_budget, slots={r: len(s) for r, s in srv.slots.items()},
                offered_frames_per_s=round(len(arr) / duration, 2), duration_s=duration,
                check="learned" if check_impl else "plain", rejected=dict(srv.rejected),
                released=dict(srv.released))
    return summ, be, fin


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--max-batch", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=96.0)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    pools = make_pools(6, 16)
    out = {}
    for ci in (0, 1):
        sur = None
        if ci:
            from paper_2504_05148_amd.train_surrogate import load_weights
            sur = load_weights()[:2]
        s, _, _ = run_serving(args.seconds, max_batch=args.max_batch,
                              hbm_budget=int(args.budget_gib * (1 << 30)), check_impl=ci,
                              surrogate=sur, pools=pools,
                              log=lambda a, b: print(f"[serving] {a}/{b}", flush=True))
        out[s["check"]] = s
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
