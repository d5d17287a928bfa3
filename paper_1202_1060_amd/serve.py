"""Request serving with continuous batching over resident codes.

A :class:`Server` owns device code tables (one :class:`Code` per resident
code, created once) and serves a stream of decode requests, each some frames
of one code. Two policies share the request bookkeeping:

* ``batched``: up to ``max_inflight`` launches are in flight, each on its
  own stream. Whenever one finishes (or at start), every request that has
  arrived and fits the device-memory budget is admitted, in arrival order,
  and all of them go out as one asynchronous ldpc_decode_batched call:
  requests of different codes and frame counts share the persistent
  workgroups, frames retire one by one at their first zero syndrome, and
  launches of consecutive admissions overlap on the device;
* ``plain``: one ldpc_decode launch per request, in arrival order on one
  stream, with FP32 messages (the reference policy).

Memory: an admitted request holds its outputs (hard decisions, iteration
count, syndrome flag, and with ``posteriors`` the total LLRs) and, when its
LLRs arrive in host memory, their device copy, until its launch completes;
the budget caps the bytes held by requests in flight. Request LLRs are
either device buffers owned by the caller or a pinned host buffer that the
server stages per launch (``Requests``); code tables and message state stay
on the device (messages live in LDS for the whole decode of a frame).

Times are host wall-clock: a request is done when the host sees the event
recorded after its launch complete; latency = done - arrival.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque

import numpy as np
import torch

from . import _native, LDPC_FLAG_EARLY_STOP, msg_flag

# ldpc_problem as a numpy record (same layout as the C struct)
PROBLEM_DTYPE = np.dtype({"names": ["code", "llr", "num_frames", "max_iter", "hard", "post", "iters", "syn_ok"],
                          "formats": [np.uint64, np.uint64, np.int32, np.int32, np.uint64, np.uint64,
                                      np.uint64, np.uint64],
                          "offsets": [0, 8, 16, 20, 24, 32, 40, 48], "itemsize": 56})
assert ctypes.sizeof(_native.ldpc_problem) == PROBLEM_DTYPE.itemsize


class Requests:
    """A request stream as arrays: arrival time (s, nondecreasing), code
    index, frame count, the request's LLRs and iteration cap.

    LLRs either sit in device memory already (``llr_addr``: device address
    of [frames][n] float32 per request) or arrive in host memory
    (``host_llr``: a pinned 1-D CPU tensor, float32 or float16, holding every
    request's [frames][n] LLRs back to back in arrival order, request i at
    elements ``host_off[i] .. host_off[i+1]``); the server then copies each
    admitted group of requests to the device with one asynchronous copy on
    its launch stream (widening 16-bit LLRs to float32 there), so staging is
    part of every request's latency."""

    def __init__(self, arrival, code, frames, llr_addr, max_iter, host_llr=None, host_off=None):
        self.arrival = np.asarray(arrival, dtype=np.float64)
        self.code = np.asarray(code, dtype=np.int64)
        self.frames = np.asarray(frames, dtype=np.int64)
        self.llr_addr = None if llr_addr is None else np.asarray(llr_addr, dtype=np.uint64)
        self.max_iter = np.asarray(max_iter, dtype=np.int32)
        self.host_llr = host_llr
        self.host_off = None if host_off is None else np.asarray(host_off, dtype=np.int64)
        assert np.all(np.diff(self.arrival) >= 0)
        assert (self.llr_addr is None) != (host_llr is None), "give llr_addr or host_llr"
        if host_llr is not None:
            assert host_llr.dim() == 1 and host_llr.dtype in (torch.float32, torch.float16)
            assert len(self.host_off) == len(self.arrival) + 1

    def __len__(self):
        return len(self.arrival)


class Server:
    def __init__(self, codes, *, policy="batched", msg="fp16", early_stop=True, budget_bytes=1 << 30,
                 max_inflight=4, device=0, posteriors=False):
        if policy not in ("batched", "plain"):
            raise ValueError(policy)
        self.codes = list(codes)
        self.policy = policy
        self.msg = "fp32" if policy == "plain" else msg
        self.flags = msg_flag(self.msg) | (LDPC_FLAG_EARLY_STOP if early_stop else 0)
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight) if policy == "batched" else 1 << 30
        self.device = torch.device("cuda", device)
        self.n = np.array([c.n for c in self.codes], dtype=np.int64)
        self.handles = np.array([c.handle for c in self.codes], dtype=np.uint64)
        nstreams = max_inflight if policy == "batched" else 1
        self.streams = [torch.cuda.Stream(self.device) for _ in range(nstreams)]
        self.lib = _native.load()
        self.posteriors = bool(posteriors)

    def request_bytes(self, req: Requests):
        """Device bytes a request holds while in flight: its outputs (hard
        decisions, iteration count, syndrome flag, and posteriors if kept)
        and, for LLRs staged from host memory, their device copy (plus the
        float32 widening of 16-bit LLRs)."""
        per_bit = 5 if self.posteriors else 1
        if req.host_llr is not None:
            per_bit += 4 if req.host_llr.dtype == torch.float32 else 6
        return req.frames * (self.n[req.code] * per_bit + 4 + 1)

    def run(self, req: Requests, *, keep_results=False, clock=time.perf_counter):
        """Serve the stream in real time; returns per-request arrays
        (done time, latency) and totals. With keep_results the outputs of
        every request are returned as host arrays (hard, iters, syn_ok)."""
        N = len(req)
        need = self.request_bytes(req)
        if N and need.max() > self.budget:
            raise ValueError("a request needs more device memory than the budget")
        done_t = np.full(N, np.nan)
        results = [None] * N if keep_results else None
        inflight = deque()  # (event, first, last, stream index, bytes, buffers)
        free_streams = deque(range(len(self.streams)))
        held = 0
        nxt = 0          # first request not yet admitted
        finished = 0
        launches = 0
        t0 = clock()
        while finished < N:
            now = clock() - t0
            # retire completed launches (in order per stream, any order overall)
            for _ in range(len(inflight)):
                ev, a, b, si, nbytes, bufs = inflight.popleft()
                if ev.query():
                    done_t[a:b] = clock() - t0
                    finished += b - a
                    held -= nbytes
                    if self.policy == "batched":
                        free_streams.append(si)
                    if keep_results:
                        self._keep(results, req, a, b, bufs)
                else:
                    inflight.append((ev, a, b, si, nbytes, bufs))
            # admit: every arrived request that fits, oldest first
            arrived = int(np.searchsorted(req.arrival, now, side="right"))
            if nxt < arrived and free_streams:
                cum = np.cumsum(need[nxt:arrived])
                take = int(np.searchsorted(cum, self.budget - held, side="right"))
                if self.policy == "plain":
                    take = min(take, 1)
                if take > 0:
                    a, b = nxt, nxt + take
                    si = free_streams.popleft() if self.policy == "batched" else 0
                    nbytes = int(cum[take - 1])
                    ev, bufs = self._launch(req, a, b, self.streams[si])
                    inflight.append((ev, a, b, si, nbytes, bufs))
                    held += nbytes
                    nxt = b
                    launches += 1
                    continue
            if not inflight and nxt < N and arrived <= nxt:
                # idle until the next arrival
                wait = req.arrival[nxt] - (clock() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        end = clock() - t0
        lat = done_t - req.arrival
        out = dict(done=done_t, latency=lat, makespan=end, launches=launches,
                   p50_ms=float(np.percentile(lat, 50) * 1e3) if N else 0.0,
                   p99_ms=float(np.percentile(lat, 99) * 1e3) if N else 0.0,
                   mean_ms=float(lat.mean() * 1e3) if N else 0.0)
        if keep_results:
            out["results"] = results
        return out

    def _launch(self, req: Requests, a: int, b: int, stream):
        F = req.frames[a:b]
        n = self.n[req.code[a:b]]
        hard_off = np.concatenate([[0], np.cumsum(F * n)])
        it_off = np.concatenate([[0], np.cumsum(F)])
        staged = None
        with torch.cuda.stream(stream):
            if req.host_llr is not None:
                # one copy of the group's LLRs (contiguous in host memory),
                # widened to float32 on the device
                h0, h1 = int(req.host_off[a]), int(req.host_off[b])
                dev_in = torch.empty(h1 - h0, dtype=req.host_llr.dtype, device=self.device)
                dev_in.copy_(req.host_llr[h0:h1], non_blocking=True)
                staged = dev_in if dev_in.dtype == torch.float32 else dev_in.float()
                llr_addr = np.uint64(staged.data_ptr()) + (4 * (req.host_off[a:b] - h0)).astype(np.uint64)
            else:
                llr_addr = req.llr_addr[a:b]
            hard = torch.empty(int(hard_off[-1]), dtype=torch.uint8, device=self.device)
            iters = torch.empty(int(it_off[-1]), dtype=torch.int32, device=self.device)
            syn = torch.empty(int(it_off[-1]), dtype=torch.uint8, device=self.device)
            post = torch.empty(int(hard_off[-1]), dtype=torch.float32, device=self.device) \
                if self.posteriors else None
        probs = np.zeros(b - a, dtype=PROBLEM_DTYPE)
        probs["code"] = self.handles[req.code[a:b]]
        probs["llr"] = llr_addr
        probs["num_frames"] = F
        probs["max_iter"] = req.max_iter[a:b]
        probs["hard"] = np.uint64(hard.data_ptr()) + hard_off[:-1].astype(np.uint64)
        probs["iters"] = np.uint64(iters.data_ptr()) + (4 * it_off[:-1]).astype(np.uint64)
        probs["syn_ok"] = np.uint64(syn.data_ptr()) + it_off[:-1].astype(np.uint64)
        if post is not None:
            probs["post"] = np.uint64(post.data_ptr()) + (4 * hard_off[:-1]).astype(np.uint64)
        if self.policy == "plain":
            p = probs[0]
            rc = self.lib.ldpc_decode(ctypes.c_void_p(int(p["code"])), ctypes.c_void_p(int(p["llr"])),
                                      int(p["num_frames"]), int(p["max_iter"]), self.flags,
                                      ctypes.c_void_p(int(p["hard"])), ctypes.c_void_p(int(p["post"]) or None),
                                      ctypes.c_void_p(int(p["iters"])),
                                      ctypes.c_void_p(int(p["syn_ok"])), ctypes.c_void_p(stream.cuda_stream))
        else:
            rc = self.lib.ldpc_decode_batched(probs.ctypes.data_as(ctypes.POINTER(_native.ldpc_problem)),
                                              b - a, self.flags, ctypes.c_void_p(stream.cuda_stream))
        _native.check(rc)
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev, (hard, iters, syn, post, hard_off, it_off, n, staged)

    @staticmethod
    def _keep(results, req, a, b, bufs):
        hard, iters, syn, post, hard_off, it_off, n, _ = bufs
        h, it, sy = hard.cpu().numpy(), iters.cpu().numpy(), syn.cpu().numpy()
        po = post.cpu().numpy() if post is not None else None
        for j in range(b - a):
            F = int(req.frames[a + j])
            results[a + j] = dict(hard=h[hard_off[j]:hard_off[j + 1]].reshape(F, int(n[j])),
                                  iters=it[it_off[j]:it_off[j + 1]], syn_ok=sy[it_off[j]:it_off[j + 1]])
            if po is not None:
                results[a + j]["post"] = po[hard_off[j]:hard_off[j + 1]].reshape(F, int(n[j]))


__all__ = ["Server", "Requests", "PROBLEM_DTYPE"]
