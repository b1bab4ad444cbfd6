"""The C-ABI library on the host: it loads, exports every declared entry
point, validates like the reference, and its host sampler (the paper's CPU
sampling step, Sec. IV-C) reproduces the reference's draws bit for bit.
No GPU call is made here."""
import os
import re

import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "aeb.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(aeb_[a-z0-9_]+)\s*\(", hdr)))


def test_every_declared_symbol_is_exported(B):
    names = declared_functions()
    assert "aeb_rollout" in names and "aeb_reduce" in names and "aeb_sample_params" in names
    L = B.lib()
    for name in names:
        assert hasattr(L, name), name


def test_exports_listed_in_binding(B):
    assert set(B.EXPORTS) <= set(declared_functions())


def test_version(B):
    assert B.lib().aeb_version() == B.ABI_VERSION


def test_validation_agrees_with_reference(B, orc):
    from test_oracle_validate import BAD
    for change in BAD:
        d = W.single(100)
        d.update(change)
        assert B.validate(d) == B.EINVAL, change
        assert B.lib().aeb_last_error().decode() != ""
    for d in (W.single(10_000), W.paper_preset(), W.sweep(n=10)[17], W.uneven_batch(5)[2]):
        assert B.validate(d) == B.OK == orc.validate(d)


@pytest.mark.parametrize("seed,sid,slot,attempt", [(42, 0, 0, 0), (7, 123456789012, 8, 5)])
def test_host_uniforms_bitwise(B, orc, seed, sid, slot, attempt):
    got = B.uniforms(seed, sid, 1000, 50_000, slot, attempt, device=False)
    want = orc.uniforms(seed, sid, 1000, 50_000, slot, attempt)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("row", range(3))
def test_host_uniforms_known_answers(B, row):
    # the library's own generator against the published Philox4x32-10 rows
    from test_oracle_rng import kat_as_uniform_call, kat_rows, kat_uniforms
    ctr, key, out = kat_rows()[row]
    seed, sid, i, slot, attempt = kat_as_uniform_call(ctr, key)
    got = B.uniforms(seed, sid, i, 1, slot, attempt, device=False).ravel()
    assert list(got) == kat_uniforms(out)


@pytest.mark.parametrize("d", [W.single(20_000), W.paper_preset(5000), W.sweep(n=3000)[37],
                               W.uneven_batch(4)[1], W.perception(20_000),
                               W.perception(5000, occlusion=("normal", 1.0, 3.0), p_dropout=0.6,
                                            confirm=4, latency=("normal", 0.0, 0.05)),
                               W.perception(3000, frame_period=0.0),
                               W.perception(3000, occlusion=("const", 1e30), horizon=1.0),
                               W.perception(2000, occlusion=("const", 33.5), frame_period=0.3,
                                            confirm=1, p_dropout=0.0),
                               W.rare_event(5000),
                               dict(W.single(3000), proposal={"mass": ("normal", 1400.0, 90.0),
                                                              "gap": ("normal", 55.0, 3.0)})])
def test_host_sampler_bitwise(B, orc, d):
    n = min(int(d["n_samples"]), 20_000)
    got = B.sample_params(d, 0, n, device=False)
    want = orc.sample(d, 0, n)
    for c in B.COLUMNS:
        assert np.array_equal(got[c].view(np.uint64), want[c].view(np.uint64)), c


@pytest.mark.parametrize("name", ["single", "paper_preset", "perception", "rare_event"])
def test_host_sampler_bitwise_full_size(B, orc, name):
    """Every sample of the sizes the GPU tests and the benchmark run: the
    grade's sine and cosine from host libm's sin and cos on both sides (a
    compiler that merged them into one sincos call once gave a different
    last bit for a few samples in a million)."""
    n = {"single": 1_048_576, "paper_preset": 350_000}.get(name, 200_000)
    d = getattr(W, name)(n)
    got = B.sample_params(d, device=False)
    want = orc.sample(d)
    for c in B.COLUMNS:
        assert np.array_equal(got[c].view(np.uint64), want[c].view(np.uint64)), c


def test_host_sampler_subrange(B, orc):
    d = W.single(10_000)
    got = B.sample_params(d, 4321, 777, device=False)
    want = orc.sample(d, 4321, 777)
    for c in B.COLUMNS:
        assert np.array_equal(got[c], want[c]), c


def test_perception_validation_agrees(B, orc):
    from test_oracle_perception import BAD
    for change in BAD:
        d = W.perception(10)
        d.update(change)
        assert B.validate(d) == B.EINVAL == orc.validate(d), change
    assert B.validate(W.perception(10)) == B.OK


def test_importance_validation_agrees(B, orc):
    from test_oracle_importance import BAD
    for change in BAD:
        d = W.paper_preset(10)
        d.update(change)
        assert B.validate(d) == B.EINVAL == orc.validate(d), change
    assert B.validate(W.rare_event(10)) == B.OK


def test_controller_validation_agrees(B, orc):
    from test_oracle_control import BAD
    for change in BAD:
        d = W.closed_loop(10)
        d.update(change)
        assert B.validate(d) == B.EINVAL == orc.validate(d), change
    assert B.validate(W.closed_loop(10)) == B.OK == orc.validate(W.closed_loop(10))


def test_perception_needs_trigger_column(B):
    cols = {c: np.zeros(10) for c in B.COLUMNS if c != "trigger"}
    with pytest.raises(B.AebError) as e:
        B.sample_params(W.perception(10), 0, 10, device=False, out=cols)
    assert e.value.code == B.EINVAL
    B.sample_params(W.single(10), 0, 10, device=False, out=cols)   # no perception: optional


def test_host_sampler_rejects_invalid(B):
    with pytest.raises(B.AebError):
        B.sample_params(dict(W.single(10), dt=0.0), 0, 10, device=False)
    with pytest.raises(B.AebError):
        B.sample_params(W.single(10), -1, 10, device=False)


def test_tune_table_validation(B, tmp_path):
    keep = B.tune_get("fp64", "stationary")
    B.tune_set("fp64", "stationary", 64, 128, 4)
    assert B.tune_get("fp64", "stationary") == (64, 128, 4, 1)
    for bad in ((48, 256, 0), (32, 512, 0), (32, 256, -1), (32, 256, 33)):
        with pytest.raises(B.AebError):
            B.tune_set("fp64", "stationary", *bad)
    with pytest.raises(B.AebError):
        B.tune_set("fp32c", "none", 128, 256, 0)     # blocks must divide the FP32 flush period
    keep_none = B.tune_get("fp64", "none")
    B.tune_set("fp64", "none", 128, 64, 0)           # FP64 also takes 128-step blocks
    assert B.tune_get("fp64", "none") == (128, 64, 0, 1)
    B.tune_set("fp64", "none", 64, 256, 4, 2)        # two samples per thread: FP64, no lead
    assert B.tune_get("fp64", "none") == (64, 256, 4, 2)
    for p, o in (("fp32c", "stationary"), ("fp64", "lead")):
        with pytest.raises(B.AebError):
            B.tune_set(p, o, 64, 256, 0, 2)
    with pytest.raises(B.AebError):
        B.tune_set("fp64", "stationary", 64, 256, 0, 3)
    B.tune_set("fp64", "none", *keep_none)
    B.tune_set("fp64", "stationary", *keep)


def test_tune_cache_load(B, tmp_path):
    keep = [B.tune_get(p, o) for p in ("fp64", "fp32c") for o in ("none", "stationary", "lead")]
    good = tmp_path / "tune.json"
    good.write_text('{"format": 1, "entries": [\n'
                    '  {"precision": 0, "obstacle": 1, "k": 16, "block": 64, "waves_per_simd": 8, "ms": 1.0},\n'
                    '  {"precision": 1, "obstacle": 0, "k": 16, "block": 128, "waves_per_simd": 0, "ms": 2.0}\n'
                    ']}\n')
    B.tune_load(str(good))
    assert B.tune_get("fp64", "stationary") == (16, 64, 8, 1)
    assert B.tune_get("fp32c", "none") == (16, 128, 0, 1)
    v2 = tmp_path / "tune2.json"
    v2.write_text('{"format": 2, "entries": [\n'
                  '  {"precision": 0, "obstacle": 1, "k": 128, "block": 256, "waves_per_simd": 4, '
                  '"samples_per_thread": 2, "ms": 1.0}\n]}\n')
    B.tune_load(str(v2))
    assert B.tune_get("fp64", "stationary") == (128, 256, 4, 2)
    bad2 = tmp_path / "bad2.json"
    bad2.write_text('{"entries": [{"precision": 0, "obstacle": 2, "k": 64, "block": 64, '
                    '"waves_per_simd": 0, "samples_per_thread": 2}]}')
    with pytest.raises(B.AebError):                  # a lead vehicle takes one sample per lane
        B.tune_load(str(bad2))
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": [{"precision": 0, "obstacle": 0, "k": 16, "block": 64, '
                   '"waves_per_simd": 0}, {"precision": 1, "obstacle": 0, "k": 48, "block": 64, '
                   '"waves_per_simd": 0}]}')
    before = B.tune_get("fp64", "none")
    with pytest.raises(B.AebError):
        B.tune_load(str(bad))
    assert B.tune_get("fp64", "none") == before      # nothing applied from a bad file
    with pytest.raises(B.AebError):
        B.tune_load(str(tmp_path / "missing.json"))
    for (p, o), t in zip([(p, o) for p in ("fp64", "fp32c") for o in ("none", "stationary", "lead")],
                         keep):
        B.tune_set(p, o, *t)
