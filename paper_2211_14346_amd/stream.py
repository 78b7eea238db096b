"""Streaming of event chunks from pinned host memory through several
analysis channels at once (the paper reads and processes many events at a
time within the memory available and overlaps reading with processing,
sections 3 and 5.1; section 6 runs the analyses of several final states over
the same events).

Two device input slots alternate: while the compute stream runs every
channel's select -> compact -> reconstruction -> compact -> device reorder on
the chunk in one slot, the copy stream fills the other slot from pinned host
memory.  HIP events order the two streams: a slot is refilled only after the
compute that read it has finished, and compute on a slot starts only after
its copy has landed.  Each channel keeps one set of counters and one cut
order for the whole stream, so the adaptive ordering (section 5.2) carries
from chunk to chunk.

Every step runs in libhf's kernels through the C ABI (binding.py); PyTorch
supplies pinned and device memory, streams and events.
"""

import numpy as np
import torch

from . import binding as B

COLS = B.DeviceEvents.COLS
PACKED_FLOAT_COLS = tuple(k for k in COLS if k not in ("lep_q", "jet_btag"))


def pack_plan(ev):
    """True when a sample can travel in the packed transfer format without
    loss: fewer than 256 leptons and jets per event, integer charges in
    [-128, 127] and integer b-tags in [0, 255] (hf_unpack_events rebuilds the
    offsets and the float columns from bytes)."""
    lc = np.diff(np.asarray(ev["lep_off"], dtype=np.int64))
    jc = np.diff(np.asarray(ev["jet_off"], dtype=np.int64))
    q = np.asarray(ev["lep_q"], dtype=np.float32)
    b = np.asarray(ev["jet_btag"], dtype=np.float32)
    return bool((lc.size == 0 or (lc.max() < 256 and jc.max() < 256)) and np.all(q == np.rint(q)) and
                np.all((q >= -128) & (q <= 127)) and np.all(b == np.rint(b)) and np.all((b >= 0) & (b <= 255)))


class HostChunk:
    """One chunk of events in pinned host memory: the ingest layout of
    include/hf.h (float32 columns, 32-bit offsets), or with packed=True (or
    "auto" when lossless) the packed transfer format: per-event object
    counts, charges and b-tags as bytes, the other columns as float32."""

    def __init__(self, ev, index_base=0, packed=False):
        self.n = int(ev["n"])
        self.index_base = int(index_base)
        self.n_lep = int(ev["lep_off"][-1])
        self.n_jet = int(ev["jet_off"][-1])
        if packed == "auto":
            packed = pack_plan(ev)
        elif packed and not pack_plan(ev):
            raise ValueError("this sample cannot be packed without loss")
        self.packed = bool(packed)
        self.t = {}
        for k in (PACKED_FLOAT_COLS if self.packed else COLS):
            self.t[k] = self._pinned(np.ascontiguousarray(ev[k], dtype=np.float32))
        if self.packed:
            self.t["lep_cnt"] = self._pinned(np.diff(np.asarray(ev["lep_off"], dtype=np.int64)).astype(np.uint8))
            self.t["jet_cnt"] = self._pinned(np.diff(np.asarray(ev["jet_off"], dtype=np.int64)).astype(np.uint8))
            self.t["lep_q8"] = self._pinned(np.asarray(ev["lep_q"], dtype=np.float32).astype(np.int8))
            self.t["jet_btag8"] = self._pinned(np.asarray(ev["jet_btag"], dtype=np.float32).astype(np.uint8))
        else:
            for k in ("lep_off", "jet_off"):
                off = np.asarray(ev[k], dtype=np.int64)
                if off[-1] >= 2 ** 31:
                    raise ValueError(f"{k}: object count too large for a chunk")
                self.t[k] = self._pinned(off.astype(np.int32))
        nv = ev.get("n_var")
        self.t["n_var"] = None if nv is None else self._pinned(np.asarray(nv, dtype=np.int16))

    def with_base(self, index_base):
        """The same pinned columns under other global event ids (the ids key
        the variation draws, so the events count as new ones)."""
        other = object.__new__(HostChunk)
        other.__dict__.update(self.__dict__)
        other.index_base = int(index_base)
        return other

    @staticmethod
    def _pinned(a):
        t = torch.empty(a.shape, dtype=torch.from_numpy(a[:0]).dtype, pin_memory=True)
        t.copy_(torch.from_numpy(a))
        return t

    @property
    def nbytes(self):
        return sum(v.numel() * v.element_size() for v in self.t.values() if v is not None)


class DeviceSlot:
    """Device buffers for one chunk of at most n_cap events, lep_cap leptons
    and jet_cap jets, and the hf_events_t that points at them."""

    def __init__(self, n_cap, lep_cap, jet_cap, with_nvar=False, device="cuda"):
        self.n_cap, self.lep_cap, self.jet_cap = int(n_cap), int(lep_cap), int(jet_cap)
        cap = {k: (self.lep_cap if k.startswith("lep_") else self.jet_cap if k.startswith("jet_") else self.n_cap)
               for k in COLS}
        self.t = {k: torch.zeros(max(1, cap[k]), dtype=torch.float32, device=device) for k in COLS}
        self.t["lep_off"] = torch.zeros(self.n_cap + 1, dtype=torch.int32, device=device)
        self.t["jet_off"] = torch.zeros(self.n_cap + 1, dtype=torch.int32, device=device)
        self.t["n_var"] = torch.zeros(max(1, self.n_cap), dtype=torch.int16, device=device) if with_nvar else None
        self.s = B.Events(n=0, index_base=0, **{k: (None if v is None else v.data_ptr()) for k, v in self.t.items()})
        self.n = 0
        self.index_base = 0
        # landing buffers of the packed transfer format (counts 16-byte aligned)
        self.p = {"lep_cnt": torch.zeros(max(16, self.n_cap), dtype=torch.uint8, device=device),
                  "jet_cnt": torch.zeros(max(16, self.n_cap), dtype=torch.uint8, device=device),
                  "lep_q8": torch.zeros(max(1, self.lep_cap), dtype=torch.int8, device=device),
                  "jet_btag8": torch.zeros(max(1, self.jet_cap), dtype=torch.uint8, device=device)}
        self.ws_unpack = B.workspace(B.lib().hf_unpack_workspace_size(self.n_cap), device)

    @property
    def ptr(self):
        import ctypes
        return ctypes.byref(self.s)

    def load(self, hc, stream):
        """Queue the copies of a host chunk into this slot on `stream`."""
        if hc.n > self.n_cap or hc.n_lep > self.lep_cap or hc.n_jet > self.jet_cap:
            raise ValueError("chunk larger than the slot")
        if (hc.t["n_var"] is None) != (self.t["n_var"] is None):
            raise ValueError("variation-count column present in one of chunk and slot only")
        with torch.cuda.stream(stream):
            for k, src in hc.t.items():
                if src is not None and src.numel():
                    dst = self.p[k] if k in self.p else self.t[k]
                    dst[:src.numel()].copy_(src, non_blocking=True)
        if hc.packed:
            B.unpack_events(hc.n, self.p["lep_cnt"], self.p["jet_cnt"], hc.n_lep, hc.n_jet, self.p["lep_q8"],
                            self.p["jet_btag8"], self.t["lep_off"], self.t["jet_off"], self.t["lep_q"],
                            self.t["jet_btag"], self.ws_unpack, stream)
        self.n = hc.n
        self.index_base = hc.index_base
        self.s.n = hc.n
        self.s.index_base = hc.index_base


class Channel:
    """One analysis channel: a cut chain ending in a reconstruction (the
    dileptonic two-neutrino solve with `reco`, the single-neutrino chi^2 with `semilep`
    and `topology`, or the dileptonic chi^2 fit with a MET split with
    `chi2`), with its counters and cut order."""

    def __init__(self, name, cuts, capacity, reco=None, semilep=None, topology="TCHAN", precision="mixed",
                 chi2=None, device="cuda"):
        if sum(x is not None for x in (reco, semilep, chi2)) != 1:
            raise ValueError("give exactly one of reco, semilep and chi2")
        self.name = name
        self.cuts = cuts
        self.n_cuts = len(cuts)
        self.cut_arr = B.cut_table(cuts)
        # user predicates (USER cuts) need the chain kernel compiled at run time
        self.compiled = B.CompiledChain(cuts) if any(c["kind"] == "USER" for c in cuts) else None
        kinds = [c["kind"] for c in cuts]
        self.reco_id = kinds.index("RECO") if "RECO" in kinds else -1
        cap = max(1, int(capacity))
        self.capacity = cap
        self.semilep = semilep is not None
        self.chi2 = chi2 is not None
        self.kind = "semilep" if self.semilep else "chi2" if self.chi2 else "quartic"
        if self.semilep:
            self.params = B.semilep_params(semilep, topology, reco_cut=self.reco_id)
            self.out = B.SemilepOutputs(cap, device=device)
            self.ws_reco = None
        elif self.chi2:
            self.params = B.chi2_params(chi2, reco_cut=self.reco_id)
            self.out = B.Chi2Outputs(cap, device=device)
            self.ws_reco = None
        else:
            self.params = B.reco_params(reco, precision=precision, reco_cut=self.reco_id)
            self.out = B.RecoOutputs(cap, device=device, want_mbb=False)
            self.ws_reco = B.workspace(B.lib().hf_ttbar_reco_workspace_size(cap), device)
        self.order = torch.arange(self.n_cuts, dtype=torch.int32, device=device)
        self.counters = torch.zeros(self.n_cuts, 3, dtype=torch.int64, device=device)
        self.survive = torch.zeros(cap, dtype=torch.uint8, device=device)
        self.idx = torch.zeros(cap, dtype=torch.int32, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.final_idx = torch.zeros(cap, dtype=torch.int32, device=device)
        self.final_count = torch.zeros(1, dtype=torch.int64, device=device)
        self.ws_sel = B.workspace(B.lib().hf_select_workspace_size(cap, self.n_cuts), device)
        self.ws_cmp = B.workspace(B.lib().hf_compact_workspace_size(cap), device)
        self.ws_cmp2 = B.workspace(B.lib().hf_compact_workspace_size(cap), device)

    def run(self, slot, stream):
        """select -> compact -> reconstruction -> compact -> reorder on the
        chunk in `slot`, queued on `stream`."""
        n = slot.n
        if self.compiled is not None:
            B.chain_select(self.compiled, slot, self.order, self.survive, self.counters, self.ws_sel, stream)
        else:
            B.select(slot, self.cut_arr, self.n_cuts, self.order, self.survive, self.counters, self.ws_sel, stream)
        B.compact(self.survive, n, self.idx, self.count, self.ws_cmp, index_base=slot.index_base, stream=stream)
        if self.semilep:
            B.semilep_reco(slot, self.idx, self.count, self.capacity, self.params, self.out, self.counters, stream)
        elif self.chi2:
            B.dilep_chi2_reco(slot, self.idx, self.count, self.capacity, self.params, self.out, self.counters,
                              stream)
        else:
            B.ttbar_reco(slot, self.idx, self.count, self.capacity, self.params, self.out, self.counters,
                         self.ws_reco, stream)
        B.compact(self.out.t["has_sol"], n, self.final_idx, self.final_count, self.ws_cmp2, d_n=self.count,
                  mapping=self.idx, stream=stream)
        B.reorder_device(self.counters, self.cut_arr, self.n_cuts, self.order, stream)

    def results(self, n):
        """Host copy of the last chunk's results (synchronises)."""
        torch.cuda.synchronize()
        S = int(self.count.item())
        F = int(self.final_count.item())
        return {"survive": self.survive[:n].cpu().numpy(), "idx": self.idx[:S].cpu().numpy(), "count": S,
                "final": self.final_idx[:F].cpu().numpy(), "reco": self.out.host(S)}


class EventStream:
    """Double-buffered streaming of host chunks through channels."""

    def __init__(self, channels, n_cap, lep_cap, jet_cap, with_nvar=False, device="cuda"):
        self.channels = list(channels)
        self.slots = [DeviceSlot(n_cap, lep_cap, jet_cap, with_nvar, device) for _ in range(2)]
        self.copy_stream = torch.cuda.Stream(device=device)
        self.compute_stream = torch.cuda.Stream(device=device)
        self.loaded = [torch.cuda.Event() for _ in range(2)]
        self.done = [torch.cuda.Event() for _ in range(2)]

    def run(self, chunks, on_chunk=None, order_log=None):
        """Stream `chunks` (HostChunk) through every channel.  on_chunk(i,
        chunk, orders) is called after chunk i has been processed, with the
        cut orders it ran under, and synchronises the device first; without
        it the loop never waits on the host.  order_log (a list) receives,
        per chunk, device copies of the channels' cut orders that chunk ran
        under, taken on the compute stream without waiting: the measured
        costs, and so the orders, differ from run to run."""
        for i, hc in enumerate(chunks):
            s = i % 2
            slot = self.slots[s]
            self.copy_stream.wait_event(self.done[s])  # the slot's previous chunk has been processed
            slot.load(hc, self.copy_stream)
            self.loaded[s].record(self.copy_stream)
            self.compute_stream.wait_event(self.loaded[s])
            orders = None
            if on_chunk is not None or order_log is not None:
                with torch.cuda.stream(self.compute_stream):
                    orders = [ch.order.clone() for ch in self.channels]
                if order_log is not None:
                    order_log.append(orders)
            for ch in self.channels:
                ch.run(slot, self.compute_stream)
            self.done[s].record(self.compute_stream)
            if on_chunk is not None:
                torch.cuda.synchronize()
                on_chunk(i, hc, [o.cpu().numpy() for o in orders])
        torch.cuda.current_stream().wait_stream(self.compute_stream)

    def reset(self):
        """Zero the counters (and the reconstruction's work statistics) and
        restore every channel's initial cut order."""
        for ch in self.channels:
            ch.counters.zero_()
            if ch.out.t.get("stats") is not None:
                ch.out.t["stats"].zero_()
            ch.order.copy_(torch.arange(ch.n_cuts, dtype=torch.int32, device=ch.order.device))
