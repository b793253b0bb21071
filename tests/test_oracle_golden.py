"""Oracle vs worked examples derived by hand from the paper's definitions.

The fixture (tests/golden/hand_examples.json) was written by hand, with each
step of the derivation recorded beside the numbers; no program produced it.
"""
import json
import os

import numpy as np
import pytest

from oracle import df_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "hand_examples.json")))["cases"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_example(case):
    nao = case["nao"]
    B = np.array(case["B"], dtype=np.float64)
    Cocc = np.array(case["Cocc"], dtype=np.float64)
    J, K, v = O.jk(B, nao, Cocc)
    np.testing.assert_array_equal(v, np.array(case["v"], dtype=float))
    np.testing.assert_array_equal(J, np.array(case["J"], dtype=float))
    np.testing.assert_array_equal(K, np.array(case["K"], dtype=float))
    # signed weight w = -1 negates D (hence J and K)
    Jm, Km, _ = O.jk(B, nao, Cocc, w=-np.ones(Cocc.shape[1]))
    np.testing.assert_array_equal(Jm, -J)
    np.testing.assert_array_equal(Km, -K)
    Cact = np.array(case["Cact"], dtype=np.float64)
    eri, _ = O.active_eri(B, nao, Cact)
    np.testing.assert_array_equal(eri, np.array(case["eri"], dtype=float))
    Cp = np.array(case["Cp"], dtype=np.float64)
    np.testing.assert_array_equal(O.papa(B, nao, Cp, Cact), np.array(case["papa"], dtype=float))
    if "Chalf" in case:
        X = O.half_transform(B, nao, np.array(case["Chalf"], dtype=float))
        np.testing.assert_array_equal(X, np.array(case["X"], dtype=float))
    # the paper's K route with gamma = D gives the same K
    np.testing.assert_allclose(O.exchange_paper_route(B, nao, O.density(Cocc)), K, rtol=0, atol=1e-12)
