"""GPU tests of the batched uneven-size launch: each field equals the same
field sampled by its own plan (bitwise), the float64 oracle (float32
tolerance), the one-field-per-launch baseline (bitwise); graph replays agree
with each other; tile shapes keep the bits, other radix orders keep the
oracle tolerance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import grf as ogrf  # noqa: E402
from oracle import spectra  # noqa: E402
from synth import uneven_fields  # noqa: E402


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1105_2737_amd as m
    return m


def small_batch(n=24, seed=3):
    fields = uneven_fields(n=n, seed=seed, sides=(64, 96, 128, 360, 512))
    fields[0]["dims"] = (1000, 1024)     # one big field
    fields[1]["dims"] = (1024, 64)
    fields[2]["cov"] = "gaussian"
    fields[3]["cov"] = "exponential"
    fields[4]["lengths"] = (2.0, 0.5)
    return fields


def test_batch_matches_plans_oracle_and_plain(grf):
    fields = small_batch()
    print("batch dims:", [f["dims"] for f in fields], flush=True)
    b = grf.Batch(fields)
    out = b.sample()
    plain = b.sample(plain=True)
    torch.cuda.synchronize()
    assert torch.equal(out, plain)
    kinds = {"matern": spectra.MATERN, "gaussian": spectra.GAUSSIAN, "exponential": spectra.EXPONENTIAL}
    for f, d in enumerate(fields):
        plan = grf.Plan(d["dims"], lengths=d["lengths"], alg=2, cov=d["cov"], sigma=d["sigma"],
                        length_scale=d["length_scale"], nu=d["nu"])
        ref = plan.sample(seed=d["seed"], batch=1)[0]
        assert torch.equal(b.field(out, f), ref), f
        if f < 8:
            o = ogrf.sample(d["dims"], d["lengths"], kinds[d["cov"]], d["sigma"], d["length_scale"], d["nu"],
                            seed=d["seed"], batch=1, alg=2)[0]
            got = b.field(out, f).double().cpu().numpy()
            assert np.abs(got - o).max() / np.abs(o).max() <= 1e-5


def test_graph_replays_agree(grf):
    b = grf.Batch(small_batch(16, seed=5))
    out = b.empty()
    b.sample(out=out)
    first = out.clone()
    scratch = torch.empty(1 << 20, device="cuda")
    for k in range(4):
        out.fill_(float("nan"))
        scratch.normal_()                      # unrelated eager work between replays
        _ = scratch.sum().item()
        b.sample(out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, first), k


def chosen_variants(path):
    """(column variant per N_1, row variant per N_2 / 2) from a tuner cache."""
    col, row = {}, {}
    for line in path.read_text().split("\n"):
        w = line.split()
        if len(w) == 7 and w[0] == "batch" and w[3] in ("col", "row"):
            (col if w[3] == "col" else row)[int(w[5])] = int(w[6])
    return col, row


def relerr(a, b):
    return float((a.double() - b.double()).abs().max() / b.double().abs().max())


def test_tuning(grf, tmp_path, monkeypatch):
    """The tuner's choices: a field whose lengths keep the plan path's radix
    order (variants 0, 1: tile shapes only) keeps its bits; another radix
    order (variants 2, 3) changes the rounding only (float32 tolerance).  A new
    batch reads the cache; corrupt and foreign lines are ignored."""
    monkeypatch.setenv("GRF_TUNE_CACHE", str(tmp_path / "tune.txt"))
    fields = small_batch(12, seed=7)
    b = grf.Batch(fields)
    ref = b.sample().clone()
    b.tune()
    got = b.sample()
    torch.cuda.synchronize()
    col, row = chosen_variants(tmp_path / "tune.txt")
    print("tuned variants:", col, row, flush=True)
    assert col and row
    for f, d in enumerate(fields):
        n1, m = d["dims"][0], d["dims"][1] // 2
        if col[n1] < 2 and row[m] < 2:
            assert torch.equal(b.field(got, f), b.field(ref, f)), f
        else:
            assert relerr(b.field(got, f), b.field(ref, f)) <= 1e-5, f
    with open(tmp_path / "tune.txt", "a") as fh:
        fh.write("gfx950 col 512 7\ngarbage\nbatch gfx942 f32 col inv 512 1\nbatch gfx950 f32 col inv 512 9\n")
    b2 = grf.Batch(fields)
    assert torch.equal(b2.sample(), got)


@pytest.mark.parametrize("var", [1, 2, 3])
def test_variants_against_oracle(grf, tmp_path, monkeypatch, var):
    """Every column and row length on variant `var` (2, 3: the other radix
    order, another number of threads per transform): the fields match the
    float64 oracle; tile shapes alone (1) keep the bits of variant 0."""
    fields = small_batch(24, seed=11)
    ref = grf.Batch(fields).sample()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cols = sorted({d["dims"][0] for d in fields})
    rows = sorted({d["dims"][1] // 2 for d in fields})
    cache = tmp_path / "tune.txt"
    cache.write_text("".join(f"batch {arch} f32 col inv {n} {var}\n" for n in cols) +
                     "".join(f"batch {arch} f32 row inv {m} {var}\n" for m in rows))
    monkeypatch.setenv("GRF_TUNE_CACHE", str(cache))
    b = grf.Batch(fields)
    out = b.sample()
    torch.cuda.synchronize()
    assert b.info() == (1, 0)
    if var == 1:
        assert torch.equal(out, ref)
    kinds = {"matern": spectra.MATERN, "gaussian": spectra.GAUSSIAN, "exponential": spectra.EXPONENTIAL}
    for f, d in enumerate(fields):
        o = ogrf.sample(d["dims"], d["lengths"], kinds[d["cov"]], d["sigma"], d["length_scale"], d["nu"],
                        seed=d["seed"], batch=1, alg=2)[0]
        got = b.field(out, f).double().cpu().numpy()
        assert np.abs(got - o).max() / np.abs(o).max() <= 1e-5, (f, d["dims"], var)


def test_one_launch_agrees_with_two_launches(grf, monkeypatch):
    """The one persistent launch (per-XCD queues, readiness counters) gives the
    same bits as the column and row passes launched one after the other, and
    no row item's wait gave up."""
    fields = small_batch(40, seed=9)
    b1 = grf.Batch(fields)
    launches, _ = b1.info()
    print(f"launches per sample: {launches}", flush=True)
    assert launches == 1
    out1 = b1.sample()
    torch.cuda.synchronize()
    assert b1.info() == (1, 0)
    monkeypatch.setenv("GRF_BATCH_LAUNCHES", "2")
    b2 = grf.Batch(fields)
    assert b2.info()[0] == 2
    out2 = b2.sample()
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)


def test_one_launch_pipeline_groups_same_bits(grf, tmp_path, monkeypatch):
    """Pipeline groups of one field each (the row items of a field queued right
    after the next field's column items) give the same bits."""
    fields = small_batch(24, seed=4)
    ref = grf.Batch(fields).sample()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = tmp_path / "tune.txt"
    cache.write_text(f"batch {arch} f32 group inv 1 1048576\n")
    monkeypatch.setenv("GRF_TUNE_CACHE", str(cache))
    b = grf.Batch(fields)
    for _ in range(3):
        out = b.sample()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        assert b.info()[1] == 0


def test_config4_full_batch(grf, monkeypatch):
    """The 4096 uneven fields of the batched workload at full size: the one
    launch equals the two-launch route bitwise, and sampled fields match the
    float64 oracle."""
    fields = uneven_fields(4096, seed=0)
    b = grf.Batch(fields)
    out = b.sample()
    torch.cuda.synchronize()
    assert b.info() == (1, 0)
    rng = np.random.default_rng(5)
    for f in sorted(int(x) for x in rng.choice(len(fields), 6, replace=False)) + [0, 4095]:
        d = fields[f]
        o = ogrf.sample(d["dims"], d["lengths"], spectra.MATERN, d["sigma"], d["length_scale"], d["nu"],
                        seed=d["seed"], batch=1, alg=2)[0]
        e = np.abs(b.field(out, f).double().cpu().numpy() - o).max() / np.abs(o).max()
        print(f"uneven field {f} {d['dims']}: {e:.3e}", flush=True)
        assert e <= 1e-5
    monkeypatch.setenv("GRF_BATCH_LAUNCHES", "2")
    b2 = grf.Batch(fields)
    out2 = b2.sample()
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
