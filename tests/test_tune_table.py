"""The measured-tuning table's host side (no GPU): a table text installs,
reads back, and resets; malformed texts are rejected without changing the
installed table.  The sweep itself needs a GPU (tests/test_gpu_tune.py)."""
import json

import pytest

TABLE = """{"format": "qdist-tune-1", "entries": [
 {"D": 3, "size_log2": 36, "share": 1, "partial_words": 1, "seg": 1024, "depth": 4, "ms": 3.5},
 {"D": 2, "size_log2": 28, "share": 16, "partial_words": 0, "seg": 512, "depth": 3, "ms": 1.0}
]}"""


@pytest.fixture(scope="module")
def Q():
    from paper_2408_10743_amd import qdist
    return qdist


def entries(Q):
    st, text = Q.qd_tune_get()
    assert st == 0
    return json.loads(text)["entries"]


def test_load_get_reset(Q):
    assert Q.qd_tune_load(TABLE) == 0
    got = entries(Q)
    assert {(e["D"], e["size_log2"], e["share"], e["partial_words"], e["seg"], e["depth"]) for e in got} == {
        (3, 36, 1, 1, 1024, 4), (2, 28, 16, 0, 512, 3)}
    assert Q.qd_tune_reset() == 0
    assert entries(Q) == []


@pytest.mark.parametrize("bad", [
    "", "{}", '{"format": "other", "entries": []}',
    TABLE.replace('"seg": 1024', '"seg": 1020'),        # not a multiple of 8
    TABLE.replace('"share": 16', '"share": 3'),              # no such sharing bucket
    TABLE.replace('"size_log2": 28', '"size_log2": 29'),     # no such size bucket
    TABLE.replace('"D": 3', '"D": 5'),                   # no such word count
    TABLE.replace('"depth": 4', '"depth": -1'),
    TABLE.replace('"partial_words": 1', '"partial_words": 2'),
    TABLE.replace('"seg": 1024, ', ''),                  # a field missing
])
def test_malformed_tables_are_rejected(Q, bad):
    assert Q.qd_tune_load(TABLE) == 0
    assert Q.qd_tune_load(bad) == Q.QD_ERR_INVALID
    assert len(entries(Q)) == 2  # unchanged
    Q.qd_tune_reset()


def test_tune_run_needs_a_gpu(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert Q.qd_tune_run(1.0)[0] == Q.QD_ERR_DEVICE
