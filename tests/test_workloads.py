"""Workload definition: the certified scene seeds (tests/golden/reachable_seeds.txt) are
reproducible from the certificate script, and excluded scenes really fail it."""
import importlib.util
import os

from paper_2510_07674_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _certificate():
    spec = importlib.util.spec_from_file_location("make_reachable_seeds",
                                                  os.path.join(HERE, "golden", "make_reachable_seeds.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_certified_seeds_reproduce(orc):
    cert = _certificate()
    for name in ("tiny", "tower4", "tower10"):
        seeds = synth.certified_seeds(name)
        assert len(seeds) >= 32 and seeds == sorted(set(seeds))
        for s in seeds[:2]:
            assert cert.certify(name, s)
        first_gap = next(s for s in range(seeds[-1]) if s not in seeds)
        assert not cert.certify(name, first_gap)
