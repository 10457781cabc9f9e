"""The learned tuner at its workload's shape, on the GPU.  Kept in a file of its
own, collected after the parity tests: its bounds are on measured times, which
vary from box to box, while every other GPU test checks exact results."""
import pytest
import torch

from paper_2007_01277_amd import hfuse as H
from paper_2007_01277_amd import learned_tuner as LT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _init():
    assert torch.cuda.is_available()
    H.hf_init()


def test_learned_tuner_at_the_workload_shape():
    """The learned tuner's workload as the bench runs it: 40 seeded pairs of the
    five data kernels, every candidate profiled twice (two independent
    measurements), the ensemble trained on 50 configurations of each training
    pair, 4-fold cross-validation by pair, top 3 of 85 profiled.  Over runs
    and evaluation seeds the tuner's choice lands 3-6 % from the exhaustive
    search's choice on the second measurement and 5-8 % on the first (where
    the exhaustive best is the minimum of 85 noisy values), against 9-13 %
    for 3 candidates profiled at random and 10-20 % for the even split on the
    first; the bounds below leave room for that spread, and the tuner must
    beat the even split and the random profiles."""
    pairs = LT.draw_pairs(40, seed=2, kmin=16, kmax=26, kinds=LT.DATA_KINDS)
    data = LT.collect(pairs, reps=10, seed=2, check=True)
    res = LT.evaluate(data, folds=4, per_pair=50, topk=3, epochs=500)
    print({k: v for k, v in res.items() if k != "per_pair"}, flush=True)
    assert res["regret_mlp_checked_mean"] <= 0.08
    assert res["regret_mlp_mean"] <= 0.11
    assert res["regret_mlp_mean"] < min(res["regret_naive_mean"], res["regret_random_mean"])
