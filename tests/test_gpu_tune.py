"""The measured tuner on the GPU: a sweep installs shapes from the candidate
sets for the buckets it reached, and distances do not change under them
(config 2 and 3 golden values, a batch of every word count)."""
import json
import os

import pytest

pytestmark = pytest.mark.gpu

from oracle import oracle as O
from paper_2408_10743_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_distances.json")))


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    st, name = qdist.qd_device_check()
    assert st == 0, name
    return qdist


def test_tune_sweep_and_results_unchanged(Q):
    st, before = Q.qd_tune_get()
    assert st == 0
    try:
        st, text = Q.qd_tune_run(20.0)
        print("tune status", st, flush=True)
        assert st in (0, Q.QD_INCOMPLETE)
        entries = json.loads(text)["entries"]
        assert entries, "no bucket measured"
        for e in entries:
            assert e["seg"] in (64, 128, 256, 512, 1024, 2048, 4096) and e["depth"] in (2, 3, 4)
            assert e["ms"] > 0
        assert json.loads(Q.qd_tune_get()[1])["entries"] == entries
        for i in range(5):
            G, f = W.config2(i)
            assert Q.qd_distance(G, f)[1] == GOLD["config2"][i]
        G, f = W.config3(0)
        st, d, w, s = Q.qd_distance_ex(G, f)
        assert st == 0 and d == GOLD["config3"][0]
        codes = [W.config1(i) for i in range(4)] + [W.config2(i) for i in range(4)]
        st, ds, _, sts, _ = Q.qd_distance_batch(codes)
        assert all(x == 0 for x in sts)
        assert ds[4:] == GOLD["config2"][:4]
        assert ds[:4] == [O.brute(O.expand(G, f))[0] for G, f in codes[:4]]
    finally:
        assert Q.qd_tune_load(before) == 0
