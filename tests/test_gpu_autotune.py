"""Autotuned launch parameters (tsk_autotune): tuning a batch fills the
handle's table, plans made afterwards use it (their workspace size follows),
the results stay the oracle's to FP64 accuracy and the tuned plan's own
results are unchanged through a save / clear / load round trip of the
JSON cache."""
import json

import numpy as np
import pytest

import synth
from helpers import np_of, to_torch, tucker_rel_diff
from oracle import recompress as RC

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def tsk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_13532_amd as m
    return m


def inputs(sums):
    out = []
    for one in sums:
        cores, factors = to_torch(one, DEV, None)
        out.append({"cores": cores, "factors": factors, "kind": "krp", "sizes": [one["ell"][0]],
                    "seed": one["omega_seed"], "coeffs": one["coeffs"]})
    return out


def test_autotune_round_trip(tsk, tmp_path):
    import torch
    sums = synth.config_batch(count=256)[::16]  # 16 sums of every mode size
    batch = inputs(sums)
    tsk.autotune_clear()
    q0, h0 = tsk.BatchRecompressor(batch)()
    torch.cuda.synchronize()
    q0 = [[np_of(q) for q in qs] for qs in q0]
    h0 = [np_of(h) for h in h0]

    tsk.autotune(batch, reps=2)
    path = tmp_path / "tune.json"
    tsk.autotune_save(path)
    table = json.loads(path.read_text())
    assert table["arch"].startswith("gfx")
    kinds = {(e["kernel"], e["param"]) for e in table["entries"]}
    assert ("krp_core_sketch", "split_target") in kinds
    assert ("krp_core_sketch", "waves_per_quadrant") in kinds
    assert ("proj_final", "split_target") in kinds
    print(f"{len(table['entries'])} tuned classes")

    br = tsk.BatchRecompressor(batch)
    q1, h1 = br()
    torch.cuda.synchronize()
    q1 = [[np_of(q) for q in qs] for qs in q1]
    h1 = [np_of(h) for h in h1]
    worst = 0.0
    for one, qa, ha, qb, hb in zip(sums, q1, h1, q0, h0):
        ref = RC.recompress(one, "krp", [one["ell"][0]], one["omega_seed"])
        d_ref = tucker_rel_diff(ha, qa, ref["H"], ref["Q"])
        d_untuned = tucker_rel_diff(ha, qa, hb, qb)
        worst = max(worst, d_ref, d_untuned)
        assert d_ref < 1e-12 and d_untuned < 1e-12, (one["dims"], d_ref, d_untuned)
    print(f"tuned vs oracle and vs untuned: worst {worst:.1e}")

    # the cache reproduces the tuned plans: same workspace, same bits
    tsk.autotune_clear()
    tsk.autotune_load(path)
    br2 = tsk.BatchRecompressor(batch)
    assert br2.ws.numel() == br.ws.numel()
    q2, h2 = br2()
    torch.cuda.synchronize()
    for ha, hb in zip(h1, h2):
        assert np.array_equal(ha, np_of(hb))
    tsk.autotune_clear()


def test_autotune_load_rejects_other_arch(tsk, tmp_path):
    path = tmp_path / "other.json"
    path.write_text('{"arch": "gfx90a", "entries": []}')
    with pytest.raises(tsk.TskError):
        tsk.autotune_load(path)
