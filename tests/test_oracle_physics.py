"""Injected-truth physics of the oracle pipeline (the paper gives no TPC
efficiency; thresholds are this implementation's, set once from the oracle)."""
import numpy as np
import pytest

import synth
import truth


@pytest.mark.parametrize("cfg,eff_all,eff_hi", [("C1", 0.97, 0.98), ("C2", 0.93, 0.98)])
def test_efficiency_clones_fakes(orc, cfg, eff_all, eff_hi):
    ev = synth.make_config(cfg)
    r = orc.track(ev, precision=32)
    e = truth.efficiency(ev, r['hit_off'], r['hit_ids'], r['sector'])
    e_hi = truth.efficiency(ev, r['hit_off'], r['hit_ids'], r['sector'], pt_min=0.3)
    assert e['eff'] >= eff_all, e
    assert e_hi['eff'] >= eff_hi, e_hi
    assert e['clone_rate'] < 0.01 and e['fake_rate'] < 0.01, e
    q = r['chi2'] / r['ndf']
    assert 0.9 < np.median(q) < 1.1


def test_fp32_and_fp64_pipelines_agree_on_physics(orc):
    ev = synth.make_config('C1')
    a = orc.track(ev, precision=32)
    b = orc.track(ev, precision=64)
    ea = truth.efficiency(ev, a['hit_off'], a['hit_ids'], a['sector'])
    eb = truth.efficiency(ev, b['hit_off'], b['hit_ids'], b['sector'])
    assert abs(ea['eff'] - eb['eff']) < 0.02
