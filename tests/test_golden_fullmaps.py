"""The stored whole-map fingerprints (tests/golden/fullmaps.json) are self-consistent and
describe the seeded workloads: every ray is counted once (Section 2, Eq. (mu_ij): in the
map, out of it, or singular), the row and column sums add up to the map's sum, and the
oracle reported its near-edge rays. No GPU needed."""
import json
import os

import pytest

from paper_1005_5198_amd import workloads as w

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullmaps.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["c1", "c2", "c2_random"])
def test_fingerprint_consistent(golden, name):
    g = golden[name]
    spec = w.config1() if name == "c1" else w.config2()
    assert g["shape"] == [spec.params["npy"], spec.params["npx"]]
    assert len(g["row_sums"]) == g["shape"][0] and len(g["col_sums"]) == g["shape"][1]
    assert sum(g["row_sums"]) == g["sum"] == sum(g["col_sums"]) == g["rays_in_map"]
    assert g["rays_in_map"] + g["rays_out"] + g["rays_singular"] == spec.n_rays
    assert len(g["sha256"]) == 64
    assert g["near_edge"] == len(g["near_edge_rays"])
    # the near-edge count is about 4e-9 of the binned rays (a few at most on these maps)
    assert g["near_edge"] <= 16
