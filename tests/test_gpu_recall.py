"""The recall protocol of Section 6 (recall of the k nearest neighbours as
tables are added) runs end to end through the library, and every family's
recall grows with the number of tables."""
import pytest

from gpu_util import dev
from paper_2503_06737_amd import recall

pytestmark = pytest.mark.gpu


def test_recall_grows_with_tables():
    dev()
    res = recall.run(nq=20, reps=1, Ls=(1, 16))
    assert set(res["results"]) == {f"{p}/{m}-{f}" for p in ("shared", "per_table")
                                   for m in ("e2lsh", "srp") for f in recall.FAMILIES}
    for name, rows in res["results"].items():
        r1, r16 = rows[0]["recall"], rows[1]["recall"]
        assert 0.0 <= r1 <= r16 <= 1.0, name
        assert r16 > 0.5, name
    sb = res["state_bytes"]
    assert sb["hcs3"] < sb["hcs2"] < sb["cs"] < sb["dense"]
