"""Host logic of the packed transfer format: a chunk is packed only when the
bytes reproduce it exactly (counts below 256, integer charges and b-tags)."""

import numpy as np

import hfgen
from paper_2211_14346_amd.stream import pack_plan


def _sample():
    return hfgen.stream_chunk(hfgen.config("hlhc50M"), 0, n=5000)[0]


def test_generated_chunks_pack():
    assert pack_plan(_sample())
    assert pack_plan(hfgen.generate("hlhc50M", n_events=0))


def test_lossy_inputs_do_not_pack():
    ev = _sample()
    b = dict(ev, jet_btag=ev["jet_btag"].copy())
    b["jet_btag"][7] = 0.7  # a continuous discriminant
    assert not pack_plan(b)
    q = dict(ev, lep_q=ev["lep_q"].copy())
    q["lep_q"][0] = 300.0
    assert not pack_plan(q)
    many = dict(ev, jet_off=ev["jet_off"].copy())
    many["jet_off"] = many["jet_off"].astype(np.int64)
    many["jet_off"][1:] += 300  # event 0 with 300 more jets (only the counts matter here)
    assert not pack_plan(many)
