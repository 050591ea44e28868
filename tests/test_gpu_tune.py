"""The plan autotuner: it chooses per pass between the compile-time kernel
and the runtime-radix kernel (radix order x values per thread), the tuned
plan still matches the float64 oracle, its choices go to the tuning cache
keyed by (arch, dtype, pass, direction, length), a new plan reads them back
(the same kernels, so the same bits), and foreign or corrupt cache lines are
ignored."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import grf as ogrf  # noqa: E402
from oracle import spectra  # noqa: E402


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("dims,alg", [((720, 90), 2), ((720, 90), 1), ((512, 512), 2), ((40, 30, 18), 2),
                                      ((2700,), 2)])
def test_tuned_plan_matches_oracle_and_cache_round_trip(grf, tmp_path, monkeypatch, dims, alg):
    from paper_1105_2737_amd import _lib as L
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("GRF_TUNE_CACHE", str(cache))
    plan = grf.Plan(dims, alg=alg, dtype=torch.float32)
    plan.tune(batch=8)
    out = plan.sample(seed=4, batch=3)
    for b in range(3):
        ref = ogrf.sample(dims, (1.0,) * len(dims), spectra.MATERN, 1.0, 0.1, 1.5, seed=4 + b, batch=1, alg=alg)[0]
        assert relerr(out[b].double().cpu().numpy(), ref) <= 1e-5
    lines = [l.split() for l in cache.read_text().splitlines()]
    assert lines and all(l[0] == "plan" and l[2] == "f32" and l[4] in ("inv", "fwd") for l in lines)
    for l in lines:
        print(" ".join(l), flush=True)
    # a second plan reads the cache: the same kernels, hence the same bits
    passes = {"col-gen": L.GRF_PASS_COL_GEN_INV, "row-c2r": L.GRF_PASS_ROW_C2R, "row-gen-c2r": L.GRF_PASS_ROW_GEN_C2R,
              "row-r2c-gen": L.GRF_PASS_ROW_R2C_GEN}
    plan2 = grf.Plan(dims, alg=alg, dtype=torch.float32)
    for l in lines:
        if l[3] in passes:
            assert plan2.tune_choice(passes[l[3]], int(l[5])) == " ".join(l[6:])
    assert torch.equal(plan2.sample(seed=4, batch=3), out)


def test_cache_ignores_foreign_and_corrupt_lines(grf, tmp_path, monkeypatch):
    from paper_1105_2737_amd import _lib as L
    cache = tmp_path / "tune.txt"
    cache.write_text("\n".join([
        "plan gfx942 f32 row-c2r inv 45 generic 8 5,3,3",          # another architecture
        "plan gfx950 f32 row-c2r inv 45 generic 8 5,3",            # radices do not multiply to 45
        "plan gfx950 f32 row-c2r inv 45 generic 6 5,3,3",          # values per thread not 4 or 8
        "plan gfx950 f32 row-c2r inv 45 fixed",                     # no compile-time kernel for 45
        "plan gfx950 f32 row-c2r inv",                              # truncated
        "garbage",
        "batch gfx950 f32 col inv 512 1",                           # another scope
    ]) + "\n")
    monkeypatch.setenv("GRF_TUNE_CACHE", str(cache))
    plan = grf.Plan((64, 90), dtype=torch.float32)
    assert plan.tune_choice(L.GRF_PASS_ROW_C2R, 45) == "default"
    ref = ogrf.sample((64, 90), (1.0, 1.0), spectra.MATERN, 1.0, 0.1, 1.5, seed=2, batch=1, alg=2)[0]
    assert relerr(plan.sample(seed=2, batch=1)[0].double().cpu().numpy(), ref) <= 1e-5
    # a valid line for this device is taken
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    with open(cache, "a") as fh:
        fh.write(f"plan {arch} f32 row-c2r inv 45 generic 4 3,5,3\n")
    plan = grf.Plan((64, 90), dtype=torch.float32)
    assert plan.tune_choice(L.GRF_PASS_ROW_C2R, 45) == "generic 4 3,5,3"
    assert relerr(plan.sample(seed=2, batch=1)[0].double().cpu().numpy(), ref) <= 1e-5
