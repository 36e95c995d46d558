"""Pin the FP64 oracle to closed forms derived from the paper's definitions
(tests/golden/closed_forms.json; Sec. III-B, IV-A..IV-D)."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


@pytest.mark.parametrize("case", GOLD["cases"], ids=[c["name"] for c in GOLD["cases"]])
def test_closed_form(case):
    fp = np.array(case["footprint"], np.float32)
    pose = np.array([case["pose"]], np.float32)
    edges = np.array(case["edges"], np.float32)
    off = np.array([0, len(edges)], np.int32)
    r = oracle.psdf(fp, pose, edges, off, eps=GOLD["eps"], eps_sat=GOLD["eps_sat"], eta=case["eta"])
    tol = case.get("phi_tol", 1e-12)
    assert abs(r["phi"][0] - case["phi"]) <= tol
    if case["grad"] is not None:
        for k, g in enumerate(case["grad"]):
            if g is not None:
                assert abs(r["grad"][0, k] - g) <= 1e-9, (k, r["grad"][0], case["grad"])
    assert r["edge"][0] == case["edge"] and r["obst"][0] == 0
    if case["pen"] is not None:
        assert r["pen"][0] == case["pen"]


def test_sign_convention():
    """Positive when separated, zero at contact, negative when overlapping (Sec. III-B)."""
    fp = np.array(GOLD["cases"][0]["footprint"], np.float32)
    edges = np.array([[-1, 0.2, 1, 0.2]], np.float32)
    off = np.array([0, 1], np.int32)
    ys = np.array([-0.5, -0.1, 0.0, 0.1, 0.15], np.float32)
    poses = np.stack([np.zeros(5), ys, np.zeros(5)], 1).astype(np.float32)
    r = oracle.psdf(fp, poses, edges, off, eta=math.inf)
    # segment at y = 0.2, robot spans [y - 0.2, y + 0.2]: gap -y below, overlap
    # resolved by the shorter of moving down y or up 0.4 - y
    np.testing.assert_allclose(r["phi"], [0.5, 0.1, 0.0, -0.1, -0.15], atol=1e-7)


def test_empty_edge_set():
    fp = np.array(GOLD["cases"][0]["footprint"], np.float32)
    r = oracle.psdf(fp, np.zeros((3, 3), np.float32), np.zeros((0, 4), np.float32),
                    np.zeros(1, np.int32))
    assert np.all(np.isinf(r["phi"])) and np.all(r["edge"] == -1) and np.all(r["grad"] == 0)


def test_nan_pose():
    fp = np.array(GOLD["cases"][0]["footprint"], np.float32)
    r = oracle.psdf(fp, np.array([[np.nan, 0, 0]], np.float32), np.array([[-1, 1, 1, 1]], np.float32),
                    np.array([0, 1], np.int32))
    assert np.isnan(r["phi"][0]) and r["edge"][0] == -1 and r["obst"][0] == -1
