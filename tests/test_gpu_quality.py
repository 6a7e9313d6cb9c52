"""The image-quality harness on the GPU path (cornell, dense instant-radiosity reference of 262,144 VPLs).

Properties, not the paper's numbers: plain instant radiosity converges to the reference as its VPL
count grows; the hybrid with the walk variant that keeps near hits after the first bounce converges
too; the hybrid with the paper's walk (every near hit discarded) keeps an error floor, the near-field
light of the second and later bounces it never deposits.
"""
import pytest

torch = pytest.importorskip("torch")

from paper_2203_11484_amd import quality, scenes  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def study():
    from paper_2203_11484_amd import vplg
    ctx = vplg.context_create(0)
    try:
        yield quality.equal_sample_study(vplg, ctx, scenes.make_scene("cornell"), counts=(1024, 5120),
                                         ref_vpls=262144, converged_vpls=65536)
    finally:
        vplg.context_destroy(ctx)


def test_reference_is_dense(study):
    assert study["reference_vpls"] == 262144
    assert study["ref_rms"] > 0


def test_plain_ir_converges(study):
    e = [r["ir"] for r in study["rows"]] + [study["converged"]["ir"]]
    assert e[0] > e[1] > e[2]
    assert e[2] < 0.2 * e[0]


def test_hybrid_with_walk_variant_converges(study):
    e = [r["walk_near1"] for r in study["rows"]] + [study["converged"]["walk_near1"]]
    assert e[0] > e[1] > e[2]
    assert e[2] < 0.2 * e[0]
    assert e[2] < 0.01 * study["ref_rms"]


def test_hybrid_with_papers_walk_keeps_an_error_floor(study):
    e0 = study["rows"][0]["paper"]
    e_conv = study["converged"]["paper"]
    assert e_conv > 0.5 * e0
    assert e_conv > 0.05 * study["ref_rms"]
    # the floor is the missing light: far above where the consistent estimators end up
    assert e_conv > 10 * study["converged"]["walk_near1"]


@pytest.fixture(scope="module")
def sweep():
    from paper_2203_11484_amd import vplg
    ctx = vplg.context_create(0)
    try:
        yield quality.sweep(vplg, ctx, scenes.make_scene("cornell"), counts=(256, 1024, 4096, 16384),
                            ref_vpls=262144)
    finally:
        vplg.context_destroy(ctx)


def test_sweep_times_and_counts(sweep):
    """Every method makes the VPLs it was asked for (Keller's schedule: at most that many) and its gather
    time grows with the count."""
    for name, d in sweep["methods"].items():
        if name in ("ir_keller", "keller"):
            assert all(0.5 * c <= n <= c for n, c in zip(d["vpls"], sweep["counts"])), (name, d["vpls"])
        else:
            assert d["vpls"] == list(sweep["counts"]), name
        assert all(t > 0 for t in d["gather_ms"] + d["gen_ms"]), name
        assert d["gather_ms"][-1] > d["gather_ms"][0], name


def test_set_sum_variant_converges(sweep):
    """Brightness summed over the stratum's patches, with the near walk hits kept after the first bounce,
    converges to the reference like plain IR."""
    e = sweep["methods"]["set_sum_walk_near1"]["rmse"]
    assert e[-1] < 0.25 * e[0]
    assert e[-1] < 0.02 * sweep["ref_rms"]


def test_equal_rmse_table(sweep):
    """Plain IR reaches every target down to 2% of the image RMS; at each target the interpolated count
    lies on the grid's span, time grows as the target falls, and the paper's walk, with its error floor,
    does not reach the lowest targets."""
    rows = quality.equal_rmse_table(sweep, fractions=(0.2, 0.1, 0.05, 0.02))
    prev = 0.0
    for r in rows:
        ir = r["methods"]["ir"]
        assert ir["vpls"] is not None and 256 <= ir["vpls"] <= 16384
        assert ir["gather_ms"] >= prev
        prev = ir["gather_ms"]
    assert rows[-1]["methods"]["paper"]["vpls"] is None
    assert rows[-1]["time_ratio_ir_over"]["paper"] is None
