"""The runners built on the library (equation of state, balance test) on
tiny systems: they run end to end on the GPU and report what they promise.
Needs an MI355X."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_1646_amd as pkg
    pkg.load()
    return pkg


def test_equation_of_state_single(gpu):
    from paper_1211_1646_amd import eos
    r = eos.equation_of_state(0.70, nx=32, equilibration=2000, production=2000, sample_every=20,
                              blocks=4)
    assert r["N"] == 1024 and r["blocks"] == 4
    assert math.isfinite(r["P"]) and 5.0 < r["P"] < 12.0 and r["P_se"] >= 0.0
    assert 0.0 < r["delta"] <= 0.5 * math.sqrt(2.0)


def test_equation_of_state_batch_matches_its_replicas(gpu):
    """The batched runner's per-phi result is the mean over that phi's
    replicas; with two packing fractions far apart the pressures are ordered
    and each carries the paper's reference where Table 2 has one."""
    from paper_1211_1646_amd import eos
    rows = eos.equation_of_state_batch([0.30, 0.70], nx=32, replicas=3, equilibration=2000,
                                       production=2000, sample_every=20, blocks=4)
    assert [r["phi"] for r in rows] == [0.30, 0.70]
    assert all(r["replicas"] == 3 and math.isfinite(r["P"]) and r["P_se"] > 0 for r in rows)
    assert rows[0]["P"] < rows[1]["P"]
    assert "paper_P" not in rows[0]     # Table 2 has no N = 32^2 column
    # a dilute fluid: close to Henderson's closed form (1 + phi^2/8) / (1 - phi)^2,
    # within the noise of 3 short replicas of 1,024 disks
    phi = 0.30
    rho = 4 * phi / math.pi
    assert abs(rows[0]["P"] / rho / ((1 + phi * phi / 8) / (1 - phi) ** 2) - 1) < 0.10


def test_shuffle_ablation_runs_the_four_cases(gpu):
    from paper_1211_1646_amd import ablation
    r = ablation.shuffle_ablation(0.70, side=32, per_case=2, equilibration=1000, production=1000,
                                  sample_every=20, blocks=2)
    cases = [(c["particle_shuffle"], c["set_shuffle"]) for c in r["cases"]]
    assert cases == [("yes", "yes"), ("yes", "no"), ("no", "yes"), ("no", "no")]
    for c in r["cases"]:
        assert math.isfinite(c["P"]) and 0.0 < c["acceptance"] < 1.0
    assert all("z" in c for c in r["cases"][1:])
    assert np.isfinite([c["P_se"] for c in r["cases"]]).all()
