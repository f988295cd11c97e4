"""Pin of the oracle's classification metrics (Section IV-A, Eq. 10-12) against a confusion matrix counted by
hand (golden/metrics_confusion.json)."""
import json
import os
from fractions import Fraction

import oracle


def test_metrics_hand_counted_confusion():
    with open(os.path.join(os.path.dirname(__file__), "golden", "metrics_confusion.json")) as fh:
        gd = json.load(fh)
    r = oracle.metrics(gd["pred"], gd["truth"])
    for k in ("tp", "tn", "fp", "fn"):
        assert r[k] == gd[k], k
    for k in ("accuracy", "tpr", "tnr"):
        assert abs(r[k] - float(Fraction(gd[k][0]))) <= 1e-15, k


def test_metrics_degenerate_classes():
    """A test set with one class only: the rate of the absent class is undefined (NaN), accuracy is not."""
    r = oracle.metrics([1, -1, 1], [1, 1, 1])
    assert abs(r["accuracy"] - 2 / 3) <= 1e-15 and abs(r["tpr"] - 2 / 3) <= 1e-15
    assert r["tnr"] != r["tnr"]
