"""The default parameters of the oracle and of the library are the values the
paper prints for its experiments (Sec. 7), read from tests/golden."""
import os

import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stereo_parameters.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_oracle_defaults_are_the_papers():
    g = _golden()
    d = oracle.DEFAULTS
    assert d["lam_ad"] == g["lambda_ad"]
    assert d["lam_c"] == g["lambda_census"]
    assert d["gamma"] == g["gamma_L"]
    assert d["eps"] == g["eps"]


def test_library_defaults_are_the_papers():
    try:
        from paper_2203_02300_amd import default_params
        p = default_params()
    except RuntimeError as e:  # library not built
        pytest.skip(str(e))
    g = _golden()
    assert p.lambda_ad == pytest.approx(g["lambda_ad"], abs=0)
    assert p.lambda_census == pytest.approx(g["lambda_census"], abs=0)
    assert p.gamma_L == pytest.approx(g["gamma_L"], rel=1e-7)
    assert p.eps == pytest.approx(g["eps"], rel=1e-7)
