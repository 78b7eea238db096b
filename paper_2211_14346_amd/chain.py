"""One chunk of the hot path: select -> compact -> kinematic reconstruction
(dileptonic ttbar, or the single-neutrino chi^2 fit of one-lepton events) ->
compact, with per-cut counters, adaptive reordering between steps and an
optional HIP-graph recording of the four calls.

PyTorch allocates the device buffers and provides the stream; every step
runs in libhf's kernels through the C ABI (binding.py).
"""

import numpy as np
import torch

from . import binding as B


class Chain:
    def __init__(self, ev, cuts, reco, precision="mixed", device="cuda", index_base=0, order=None,
                 schedule="auto", semilep=None, topology="TCHAN", chi2=None, segment_at=None):
        """reco: dileptonic reconstruction parameters (hfgen reco dict); or
        None with semilep (hfgen semilep dict) and topology for the
        single-neutrino reconstruction; or None with chi2 (hfgen chi2 dict)
        for the dileptonic chi^2 fit with a MET split.  segment_at=s runs
        the cuts at order positions [0, s) over all events, compacts, and
        the rest over the compacted survivors (section 5.2: heavy cuts late
        see fewer events; here they also run on densely packed wavefronts)."""
        self.device = device
        self.cuts = cuts
        self.n_cuts = len(cuts)
        self.cut_arr = B.cut_table(cuts)
        # user predicates (USER cuts) need the chain kernel compiled at run time
        self.compiled = B.CompiledChain(cuts) if any(c["kind"] == "USER" for c in cuts) else None
        kinds = [c["kind"] for c in cuts]
        self.reco_id = kinds.index("RECO") if "RECO" in kinds else -1
        self.dev = B.DeviceEvents(ev, device=device, index_base=index_base)
        n = self.dev.n
        self.n = n
        self.semilep = semilep is not None
        self.chi2 = chi2 is not None
        if self.chi2:
            self.params = B.chi2_params(chi2, reco_cut=self.reco_id)
            self.want_mbb = False
        elif self.semilep:
            self.params = B.semilep_params(semilep, topology, reco_cut=self.reco_id)
            self.want_mbb = False
        else:
            self.params = B.reco_params(reco, precision=precision, reco_cut=self.reco_id, schedule=schedule)
            self.want_mbb = bool(reco.get("want_mbb", 0))
            if self.want_mbb:
                self.params.want_mbb = 1
        self.order_host = list(range(self.n_cuts)) if order is None else list(order)
        self.order = torch.tensor(self.order_host, dtype=torch.int32, device=device)
        self.counters = torch.zeros(self.n_cuts, 3, dtype=torch.int64, device=device)
        self.survive = torch.zeros(max(n, 1), dtype=torch.uint8, device=device)
        self.idx = torch.zeros(max(n, 1), dtype=torch.int32, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.final_idx = torch.zeros(max(n, 1), dtype=torch.int32, device=device)
        self.final_count = torch.zeros(1, dtype=torch.int64, device=device)
        if self.chi2:
            self.out = B.Chi2Outputs(n, device=device)
            self.ws_reco = None
        elif self.semilep:
            self.out = B.SemilepOutputs(n, device=device)
            self.ws_reco = None
        else:
            self.out = B.RecoOutputs(n, device=device, want_mbb=self.want_mbb)
            self.ws_reco = B.workspace(B.lib().hf_ttbar_reco_workspace_size(n), device)
        self.ws_sel = B.workspace(B.lib().hf_select_workspace_size(n, self.n_cuts), device)
        self.segment_at = segment_at
        if segment_at is not None:
            if not 0 <= segment_at <= self.n_cuts:
                raise ValueError("segment_at outside [0, n_cuts]")
            self.seg_idx = torch.zeros(max(n, 1), dtype=torch.int32, device=device)
            self.seg_count = torch.zeros(1, dtype=torch.int64, device=device)
            self.seg_survive = torch.zeros(max(n, 1), dtype=torch.uint8, device=device)
            self.ws_seg = B.workspace(B.lib().hf_compact_workspace_size(n), device)
        self.ws_cmp = B.workspace(B.lib().hf_compact_workspace_size(n), device)
        self.ws_cmp2 = B.workspace(B.lib().hf_compact_workspace_size(n), device)
        self.graph = None

    # -------------------------------------------------------------- stages
    def run_select(self, stream=None):
        if self.segment_at is not None:
            return self._run_segments(stream)
        if self.compiled is not None:
            B.chain_select(self.compiled, self.dev, self.order, self.survive, self.counters, self.ws_sel, stream)
        else:
            B.select(self.dev, self.cut_arr, self.n_cuts, self.order, self.survive, self.counters, self.ws_sel,
                     stream)

    def _run_segments(self, stream=None):
        s = self.segment_at
        B.select_segment(self.dev, self.cut_arr, self.n_cuts, self.order, 0, s, self.survive, self.counters,
                         self.ws_sel, chain=self.compiled, stream=stream)
        B.compact(self.survive, self.n, self.seg_idx, self.seg_count, self.ws_seg, index_base=self.dev.index_base,
                  stream=stream)
        B.select_segment(self.dev, self.cut_arr, self.n_cuts, self.order, s, self.n_cuts, self.seg_survive,
                         self.counters, self.ws_sel, idx=self.seg_idx, count=self.seg_count, capacity=self.n,
                         chain=self.compiled, stream=stream)

    def run_compact(self, stream=None):
        if self.segment_at is not None:
            # survivors of the second segment, carried through the first one's ids
            B.compact(self.seg_survive, self.n, self.idx, self.count, self.ws_cmp, d_n=self.seg_count,
                      mapping=self.seg_idx, stream=stream)
            return
        B.compact(self.survive, self.n, self.idx, self.count, self.ws_cmp, index_base=self.dev.index_base,
                  stream=stream)

    def run_reco(self, stream=None):
        if self.chi2:
            B.dilep_chi2_reco(self.dev, self.idx, self.count, self.n, self.params, self.out, self.counters, stream)
        elif self.semilep:
            B.semilep_reco(self.dev, self.idx, self.count, self.n, self.params, self.out, self.counters, stream)
        else:
            B.ttbar_reco(self.dev, self.idx, self.count, self.n, self.params, self.out, self.counters,
                         self.ws_reco, stream)

    def run_final(self, stream=None):
        B.compact(self.out.t["has_sol"], self.n, self.final_idx, self.final_count, self.ws_cmp2, d_n=self.count,
                  mapping=self.idx, stream=stream)

    def run_reorder(self, stream=None):
        """New cut order from the accumulated counters, computed on the device."""
        B.reorder_device(self.counters, self.cut_arr, self.n_cuts, self.order, stream)

    def step(self, stream=None, reorder=False):
        """select -> compact -> reconstruction -> compact; with reorder=True also
        the device-side reordering, so that the next step runs the new order."""
        self.run_select(stream)
        self.run_compact(stream)
        self.run_reco(stream)
        self.run_final(stream)
        if reorder:
            self.run_reorder(stream)

    # -------------------------------------------------------------- graph
    def capture(self, reorder=False):
        """Record one step into a HIP graph (torch.cuda.CUDAGraph); with
        reorder=True the step ends with the device-side reordering."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        order0 = self.order.clone()
        with torch.cuda.stream(s):
            self.step(s, reorder=reorder)  # warm-up outside the graph (kernel loading)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.order.copy_(order0)  # the warm-up must not change the order
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step(reorder=reorder)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    # -------------------------------------------------------------- host side
    def counters_host(self):
        return self.counters.cpu().numpy().astype(np.uint64)

    def reorder(self):
        """New order from the accumulated counters (host), written to the
        device order buffer that the recorded graph reads."""
        new = B.reorder_stats(self.counters_host(), self.cut_arr, self.n_cuts)
        self.order_host = new
        self.order.copy_(torch.tensor(new, dtype=torch.int32), non_blocking=False)
        return new

    def reset_counters(self):
        self.counters.zero_()

    def results(self):
        torch.cuda.synchronize()
        S = int(self.count.item())
        F = int(self.final_count.item())
        out = self.out.host(S)
        idx = self.idx[:S].cpu().numpy()
        if self.segment_at is not None:  # the chain's survive mask, rebuilt from the survivors' ids
            survive = np.zeros(self.n, dtype=np.uint8)
            survive[idx - self.dev.index_base] = 1
        else:
            survive = self.survive[:self.n].cpu().numpy()
        return {"survive": survive, "idx": idx,
                "count": S, "final": self.final_idx[:F].cpu().numpy(), "reco": out,
                "counters": self.counters_host()}
