"""The benchmark modes of Sec. V on the GPU path, at the information-sharing
workload's full size (256 PEs x 4096 particles, 512 x 512 frames).

Directional claims of Sec. V-B / Fig. 3: with the randomized ring and the
adaptive ratio, every PE's estimate reaches the object in fewer iterations
than with the fixed ring (10% and 50% exchange), and without exchange some PEs
never do.  Exact curves are not pinned (the figures are not available).
"""
import numpy as np
import pytest

from paper_1310_4624_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def seq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return synth.make_sequence("arna_infoshare_512_256x4096", seed=1000, frames=40)


def test_arna_shares_information_faster_than_rna(seq):
    from paper_1310_4624_amd.experiments import infoshare
    res = {m: infoshare(m, seq=seq, steps=40) for m in ("arna", "rna10", "rna50", "rna0")}
    a = res["arna"]["converged_at"]
    assert a is not None and a <= 12, res["arna"]["converged_at"]
    for m in ("rna10", "rna50"):
        r = res[m]["converged_at"]
        assert r is None or r > a, (m, r, a)
        # after the same number of iterations fewer RNA PEs are on the object
        assert res[m]["fraction_within"][a - 1] < 1.0
    assert res["rna0"]["converged_at"] is None
    # the adaptive ratio starts at the initial 10% and then follows Eq. 3
    assert res["arna"]["n_ex"][0] == 409
    assert max(res["arna"]["n_ex"][1:4]) > 409          # one PE holds the mass: near N_p/2
    assert res["arna"]["pe_eff_over_m"][-1] > res["arna"]["pe_eff_over_m"][0]


def test_tracking_all_modes_follow_the_spots():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1310_4624_amd.experiments import tracking
    seq = synth.make_sequence("arna_tracking_512_4x64x4096", seed=1000, frames=40)
    for m in ("arna", "rna10"):
        r = tracking(m, seq=seq, steps=40)
        assert r["rmse"] < 0.8, r
        assert max(r["rmse_per_spot"]) < 1.2, r


def test_information_sharing_median_ordering():
    """The stored study (results/infoshare_256x4096.json: median over 10
    seeds of the iterations until every PE estimate is within 2 px, Sec. V-B)
    says ARNA < RNA-50% <= RNA-10% and RNA-0% never; a smaller rerun on
    three of its seeds keeps that order of medians."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import json
    import os
    from paper_1310_4624_amd.experiments import infoshare_study
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    stored = json.load(open(os.path.join(root, "results", "infoshare_256x4096.json")))
    s = stored["summary"]
    assert s["arna"]["median_converged_at"] < s["rna50"]["median_converged_at"]
    assert s["rna50"]["median_converged_at"] <= s["rna10"]["median_converged_at"]
    assert s["rna0"]["converged_runs"] == 0
    r = infoshare_study(seeds=3, modes=("arna", "rna10", "rna0"), steps=40, curve_pes=())
    m = r["summary"]
    print(m, flush=True)
    assert m["arna"]["median_converged_at"] is not None
    assert m["rna10"]["median_converged_at"] is None or (
        m["arna"]["median_converged_at"] < m["rna10"]["median_converged_at"])
    assert m["rna0"]["converged_runs"] == 0
    # the same seeds give the stored runs' convergence iterations
    for mode in ("arna", "rna10"):
        got = [x["converged_at"] for x in r["runs"][mode]]
        want = [x["converged_at"] for x in stored["runs"][mode][:3]]
        assert got == [w if w is not None and w <= 40 else None for w in want], (mode, got, want)
