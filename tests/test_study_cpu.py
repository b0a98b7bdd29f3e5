"""Host-side pieces of the ablation / sweep study (no GPU)."""
import math

import numpy as np

from paper_2602_15838_amd import study


def test_fit_exponent_recovers_power_law():
    n = np.array([2, 4, 8, 16, 32, 64, 128], np.float64)
    for e in (1.0, 1.2, 2.5):
        assert abs(study.fit_exponent(n, 3.7 * n ** e) - e) < 1e-12


def test_variants_are_the_paper_ablation():
    """base = nothing reused; hotstart = previous iterate and factors reused;
    turbo = hotstart plus the Riccati warm start of the first iteration."""
    v = study.VARIANTS
    assert v["base"] == dict(cache_factors=False, riccati_warmstart=False, hotstart=False)
    assert v["hotstart"] == dict(cache_factors=True, riccati_warmstart=False, hotstart=True)
    assert v["turbo"] == dict(cache_factors=True, riccati_warmstart=True, hotstart=True)
    assert study.ABLATION_AGENTS == (2, 4, 6, 10, 14)


def test_study_scenarios_shapes():
    p, scs = study.ablation_scenarios(6, 3)
    assert p.dp == 2 and len(scs) == 3 and all(s.N == 6 and s.T == 20 for s in scs)
    assert not np.allclose(scs[0].starts, scs[1].starts)      # seeds differ
    p3, sc = study.sweep_scenario(32)
    assert p3.dp == 3 and sc.N == 32 and sc.T == 50
    r = np.linalg.norm(sc.starts, axis=1)
    np.testing.assert_allclose(r, 12.0 * math.sqrt(32 / 128), rtol=1e-12)
