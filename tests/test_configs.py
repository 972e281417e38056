"""The workload descriptions under configs/ agree with the generator's own
configurations, so the files cannot drift from what the tests and the
benchmark run (CPU only)."""
import os

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load(name):
    return synth.load_config_file(os.path.join(ROOT, "configs", f"{name}.json"))


def test_config0_and_1_systems():
    assert load("config0")["systems"] == [synth.config0()]
    assert load("config1")["systems"] == [synth.config1()]
    assert load("config2")["systems"] == [synth.config1()]


def test_config3_systems():
    assert load("config3")["systems"] == synth.config3_systems()
    assert load("config3")["rhs"]["per_system"] == 32


def test_config4_families():
    d = load("config4")
    train, held = d["families"]["train"], d["families"]["held_out"]
    assert len(train) == 200 and len(held) == 20
    assert sum(c.nx == 16 for c in train) == 160 and sum(c.nx == 80 for c in train) == 40
    assert all(c.nx == 80 for c in held)
    assert all(30 <= c.n_stations <= 229 and 0.05 <= c.damp <= 0.5 for c in train + held)
    seeds = {c.seed for c in train}
    assert not seeds & {c.seed for c in held}
    assert train == synth.c17_family("cfg0", 1, 160) + synth.c17_family("cfg1", 161, 40)


def test_every_config_states_its_readings():
    for k in range(5):
        d = load(f"config{k}")
        assert d["name"] == f"config{k}"
        for key in ("description", "solver", "parity", "readings"):
            assert d[key], (k, key)
        for key in ("operator", "stopping", "jacobi", "scalar_rounding"):
            assert key in d["readings"], (k, key)


def test_unknown_family_rejected(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text('{"name": "x", "families": {"train": [{"family": "other"}]}}')
    with pytest.raises(ValueError):
        synth.load_config_file(str(p))
