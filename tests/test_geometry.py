"""Host-side geometry and accounting, pinned to the numbers the paper prints."""
import json
import os

import pytest

from paper_1412_2629_amd import geometry as G

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_flop_counts():
    g = GOLD["flops"]
    assert G.PAPER_DW_FLOPS == g["dw"] and G.CLOVER_FLOPS == g["clover"] and G.PAPER_A_FLOPS == g["A"]
    assert G.PAPER_DW_FLOPS + G.CLOVER_FLOPS == G.PAPER_A_FLOPS
    assert G.DSLASH_FLOPS == 1320 and G.A_FLOPS == 1824


def test_working_set():
    g = GOLD["working_set_kB"]
    sp = G.domain_working_set(g["domain"], 4, 4)
    assert sp["spinors"] == 7 * g["half_spinor"] * 1024
    assert sp["links"] == g["links_sp"] * 1024 and sp["clover"] == g["clover_sp"] * 1024
    assert sp["total"] == g["total_sp"] * 1024
    hp = G.domain_working_set(g["domain"], 4, 2)
    assert hp["links"] == g["links_hp"] * 1024 and hp["clover"] == g["clover_hp"] * 1024


def test_load_examples():
    g = GOLD["load_examples"]
    c0, c1, c2 = g["cases"]
    assert round(G.load(c0["n_domain"], c0["n_core"]), 2) == c0["load"]
    nd = G.n_domain(G.volume(c1["local_volume"]), 512)
    assert nd == c1["n_domain"] and G.load(nd, c1["n_core"]) == c1["load"]
    nd = G.n_domain(G.volume(c2["global"]) // c2["nodes"], 512)
    assert nd == c2["n_domain"] and round(G.load(nd, c2["n_core"]), 2) == c2["load"]
    nu = g["non_uniform"]
    n = len(nu["domains"])
    assert round(sum(nu["domains"]) / (n * nu["n_core"]), 2) == nu["load"]


@pytest.mark.parametrize("row", GOLD["table3"]["rows"])
def test_table3_load(row):
    L, knc, nd_want, load_pct = row
    nd = G.n_domain(G.volume(L) // knc, 512)
    assert nd == nd_want
    assert round(100 * G.load(nd, 60)) == load_pct


def test_domain_checks():
    assert G.check_domains((16, 16, 16, 32), (8, 4, 4, 4))
    assert not G.check_domains((8, 8, 8, 8), (8, 4, 4, 4))            # one domain in x
    assert not G.check_domains((24, 24, 24, 48), (8, 4, 4, 4))        # three domains in x
    assert G.check_domains((12, 12, 12, 24), (2, 2, 2, 2))
    assert not G.check_domains((12, 12, 12, 24), (4, 4, 4, 4))


def test_hop_counts():
    b = (8, 4, 4, 4)
    assert G.in_domain_hops(b) + G.face_hops(b) == 8 * 512
    assert G.face_hops(b) == 2 * (64 + 3 * 128)
    b = (2, 2, 2, 2)
    assert G.in_domain_hops(b) == G.face_hops(b) == 64
