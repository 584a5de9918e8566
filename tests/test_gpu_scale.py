"""The 1e6-lens scale of Section 2's Phi_fiducial (2500^2 pixels, 3.1e15 interactions) on the
HIP path (needs an MI355X): sampled rays of the full geometry against the FP64 oracle, and one
band of rows made in the launch configuration the benchmark times."""
import sys

import numpy as np
import pytest

import oracle
from paper_1005_5198_amd import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1005_5198_amd as rs_mod
    oracle.build(force=False)
    return rs_mod


@pytest.fixture(scope="module")
def spec():
    return w.phi_fiducial()


def test_phi_fiducial_sampled_rays_match_oracle(rs, spec):
    """64 x 32-ray windows (one deflection block each) at seeded places, every ray against the
    oracle's 1e6-lens FP64 sum: mixed mode exact; the FP32 changed-ray fraction is reported."""
    xy, _ = rs.lens_tensors(spec.lens_xy)
    rng = np.random.default_rng(66)
    changed = total = 0
    for _ in range(3):
        i0 = int(rng.integers(0, spec.params["nx"] - 64))
        j0 = int(rng.integers(0, spec.params["ny"] - 32))
        sub = spec.window(i0, i0 + 64, j0, j0 + 32)
        say("phi_fiducial window", i0, j0)
        pix_o, _, _ = oracle.ray_pixels(sub.params, sub.lens_xy)
        pix_m = rs.ray_pixels(sub.params, xy, None, mode="mixed").cpu().numpy().astype(np.int64)
        assert np.array_equal(pix_m, pix_o), f"{int(np.count_nonzero(pix_m != pix_o))} rays differ"
        pix_f = rs.ray_pixels(sub.params, xy, None, mode="fp32").cpu().numpy().astype(np.int64)
        changed += int(np.count_nonzero(pix_f != pix_o))
        total += len(pix_o)
    say(f"  fp32 changed-ray fraction at 1e6 lenses: {changed / total:.3e}")


def test_phi_fiducial_band_conserves_rays(rs, spec):
    from paper_1005_5198_amd import bench_extra
    r = bench_extra.phi_fiducial(rs, rows=32)
    say("phi_fiducial band:", {k: r[k] for k in ("rate", "pct_fp32_peak", "recheck_fraction", "projected_full_map_s")})
    assert r["rays"] == 32 * spec.params["nx"]
    assert r["recheck_fraction"] < 0.5
