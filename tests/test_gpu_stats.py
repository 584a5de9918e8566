"""Map statistics on the HIP path vs the oracle (needs an MI355X).

Inputs: seeded synthetic count-map pairs (one magnification field, two
independent Poisson drawings, with empty pixels and caustic spikes whose counts
exceed the kernel's on-chip histogram range), and maps the oracle and the HIP
path each compute from the same lenses.

Tolerances, from the FP64 arithmetic:
  * counts, histograms, maxima, empty pixels, n_both: exact (integer work);
  * dm per pixel: the device and host log10 each round to within 1 ulp, so
    |dm_gpu - dm_oracle| <= 4 ulp(|dm|) (plus 1e-300 for dm = 0);
  * D: the same two empirical-CDF values are differenced on both sides, but the
    maximising pair can be formed from complementary counts (the oracle works
    with dm, the kernel with mu), so D agrees to 2 ulp(1) = 4.5e-16;
  * RMS: each term carries about 2.5 * 2 ulp(|log10 mu|) of log rounding and the
    sums run in different orders over at most 2^24 terms, so the relative
    difference is below n 2^-53 + 1e-13 <= 2e-9;
  * P(KS): a smooth function of D (slope <= 1.1 sqrt(n_e)) evaluated with
    device exp, so |dP| <= 1e-11 at these sizes;
  * mean mu: one division of an exact integer sum vs numpy's mean of quotients,
    relative 1e-12.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import stats as S
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_pair(rs, a, b, nr_a, nr_b, label):
    say("compare", label, a.shape, "nr", nr_a, nr_b, "max", int(a.max()), int(b.max()))
    ref = S.compare_maps(a, b, nr_a, nr_b)
    got = rs.compare_maps(dev(a), dev(b), nr_a, nr_b)
    assert got["n_pix"] == a.size
    assert got["max_a"] == ref["max_a"] and got["max_b"] == ref["max_b"]
    assert got["n_zero_a"] == ref["n_zero_a"] and got["n_zero_b"] == ref["n_zero_b"]
    assert got["n_both"] == ref["n_both"]
    assert got["ks_d"] == pytest.approx(ref["ks_d"], abs=4.5e-16)
    assert got["ks_p"] == pytest.approx(ref["ks_p"], abs=1e-11)
    if math.isnan(ref["rms_dm"]):
        assert math.isnan(got["rms_dm"])
    else:
        assert got["rms_dm"] == pytest.approx(ref["rms_dm"], rel=2e-9, abs=1e-13)
    assert got["mean_mu_a"] == pytest.approx(ref["mean_mu_a"], rel=1e-12)
    assert got["mean_mu_b"] == pytest.approx(ref["mean_mu_b"], rel=1e-12)
    say("  rms", got["rms_dm"], "D", got["ks_d"], "P", got["ks_p"])
    return got, ref


# (ny, nx, N_rays a, N_rays b, seed): ragged sizes (not a multiple of 4 or of
# the pass's block coverage), equal and doubled N_rays, low N_rays with many
# empty pixels, high N_rays whose spikes pass the on-chip bins.
PAIRS = [
    (257, 263, 4.0, 4.0, 11),
    (1024, 1024, 2.44140625, 4.8828125, 12),
    (999, 1001, 100.0, 100.0, 13),
    (2048, 2048, 500.0, 1000.0, 14),
    (1, 3, 2.0, 2.0, 15),
]


@pytest.mark.parametrize("ny,nx,nr_a,nr_b,seed", PAIRS)
def test_compare_matches_oracle(rs, ny, nx, nr_a, nr_b, seed):
    a, b = w.count_map_pair(ny, nx, nr_a, nr_b, seed)
    check_pair(rs, a, b, nr_a, nr_b, f"pair seed {seed}")


def test_compare_at_4096_squared(rs):
    """The paper's largest map size (4096^2 pixels), N_rays = 500 against 1000."""
    a, b = w.count_map_pair(4096, 4096, 500.0, 1000.0, 16, spike_frac=2e-4)
    check_pair(rs, a, b, 500.0, 1000.0, "4096^2")


def test_compare_degenerate(rs):
    ones = np.ones((64, 64), np.uint32)
    got, _ = check_pair(rs, ones, ones, 1.0, 1.0, "identical")
    assert got["rms_dm"] == 0.0 and got["ks_d"] == 0.0 and got["ks_p"] == 1.0
    got, _ = check_pair(rs, ones, 100 * ones, 1.0, 1.0, "disjoint")
    assert got["ks_d"] == 1.0 and got["rms_dm"] == pytest.approx(5.0, rel=1e-15)
    zeros = np.zeros((8, 8), np.uint32)
    got, _ = check_pair(rs, zeros, ones[:8, :8], 1.0, 1.0, "all empty")
    assert math.isnan(got["rms_dm"]) and got["n_both"] == 0 and got["ks_d"] == 1.0


def test_compare_unaligned_maps(rs):
    """Views starting one element in (not 16-byte aligned) take the scalar path, same results."""
    a, b = w.count_map_pair(300, 301, 20.0, 20.0, 17)
    fa, fb = dev(np.concatenate([[7], a.ravel()]).astype(np.uint32)), dev(np.concatenate([[9], b.ravel()]).astype(np.uint32))
    ref = S.compare_maps(a, b, 20.0, 20.0)
    got = rs.compare_maps(fa[1:], fb[1:], 20.0, 20.0)
    assert got["ks_d"] == pytest.approx(ref["ks_d"], abs=4.5e-16)
    assert got["rms_dm"] == pytest.approx(ref["rms_dm"], rel=2e-9)
    assert got["n_both"] == ref["n_both"] and got["max_b"] == ref["max_b"]


def test_compare_rejects_a_low_bound(rs):
    from paper_1005_5198_amd._lib import RayshootError
    a, b = w.count_map_pair(128, 128, 50.0, 50.0, 18)
    with pytest.raises(RayshootError, match="exceeds its bound"):
        rs.compare_maps(dev(a), dev(b), 50.0, 50.0, max_a=int(a.max()) - 1)
    with pytest.raises((RayshootError, ValueError)):
        rs.compare_maps(dev(a), dev(b), -1.0, 50.0)


@pytest.mark.parametrize("seed,max_count", [(21, None), (22, 30), (23, 5000)])
def test_histogram_matches_oracle(rs, seed, max_count):
    a, _ = w.count_map_pair(517, 389, 40.0, 40.0, seed)
    mc = int(a.max()) if max_count is None else max_count
    got = rs.histogram(dev(a), mc).cpu().numpy()
    assert np.array_equal(got, S.histogram(a, mc))


def test_map_max_and_delta_m_match_oracle(rs):
    a, _ = w.count_map_pair(701, 333, 3.0, 3.0, 31)
    assert rs.map_max(dev(a)) == int(a.max())
    got = rs.delta_m(dev(a), 3.0).cpu().numpy()
    ref = S.delta_m(a, 3.0)
    inf = np.isinf(ref)
    assert np.array_equal(np.isinf(got), inf) and np.all(got[inf] > 0)
    tol = 4 * np.spacing(np.abs(ref[~inf])) + 1e-300
    assert np.all(np.abs(got[~inf] - ref[~inf]) <= tol)


def test_rays_per_pixel_matches_oracle(rs):
    for spec in (w.config0(), w.config1(), w.config2()):
        assert rs.rays_per_pixel(spec.params) == pytest.approx(S.rays_per_pixel(spec.params), rel=1e-15)


def test_map_pipeline_matches_oracle(rs):
    """Two maps of the same lenses at N_rays = 4 and 16 (the config0 field): each side makes
    its own maps (oracle: FP64 definition; HIP: mixed mode) and its own statistics."""
    s4 = w.config0()
    p16 = dict(s4.params)
    p16.update(nx=2048, ny=2048, i1=2048, j1=2048)
    say("pipeline: oracle maps")
    m4, _ = oracle.make_map(s4.params, s4.lens_xy, s4.lens_m)
    m16, _ = oracle.make_map(p16, s4.lens_xy, s4.lens_m)
    nr4, nr16 = S.rays_per_pixel(s4.params), S.rays_per_pixel(p16)
    ref = S.compare_maps(m4, m16, nr4, nr16)
    say("pipeline: HIP maps")
    g4 = rs.make_map(s4.params, s4.lens_xy, s4.lens_m, mode="mixed")
    g16 = rs.make_map(p16, s4.lens_xy, s4.lens_m, mode="mixed")
    got = rs.compare_maps(g4.view(-1), g16.view(-1), rs.rays_per_pixel(s4.params), rs.rays_per_pixel(p16))
    assert got["ks_d"] == pytest.approx(ref["ks_d"], abs=4.5e-16)
    assert got["ks_p"] == pytest.approx(ref["ks_p"], abs=1e-11)
    assert got["rms_dm"] == pytest.approx(ref["rms_dm"], rel=2e-9)
    assert got["n_both"] == ref["n_both"] and got["max_a"] == ref["max_a"]
    say("  rms", got["rms_dm"], "D", got["ks_d"], "P", got["ks_p"])
