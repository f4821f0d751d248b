"""Kidnapping-style spreading over identical storeys (a robustness demo of the
multi-modal particle set, Sec. IV-A): particles start on every storey; while
the scans cannot tell the storeys apart, pruning keeps all of them populated,
and once a feature of the true storey comes into view the weight moves
there and the representative follows."""

import numpy as np
import pytest

from paper_2504_18056_amd import abi
from synth import configs

import bench

pytestmark = pytest.mark.gpu


def test_pruning_keeps_storeys_until_evidence_then_converges():
    c = configs.repeated_floors(N=20000)
    mass, share, best = bench.floors_run(c, abi.RESAMPLE_PRUNE)
    s = bench.floors_summary(c, mass, share, best)
    print("repeated floors (pruning):", s)
    fs = c["first_seen"]
    # Identical storeys: every storey keeps particles before the evidence.
    assert np.all(share[:fs] >= 0.05), share[:fs].min(axis=0)
    assert s["true_floor_mass_end"] > 0.95
    assert s["representative_on_true_floor_end"]
