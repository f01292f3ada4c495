"""Host-side checks of the pruner's calibration logic (no GPU)."""
import numpy as np

import paper_1611_01642_amd as pd
from oracle import pruner_oracle as P
from paper_1611_01642_amd import pruner_train as T


def _boxes(rows):
    b = np.zeros(len(rows), dtype=pd.BOX_DTYPE)
    for k, (x0, y0, x1, y1) in enumerate(rows):
        b[k]["x0"], b[k]["y0"], b[k]["x1"], b[k]["y1"] = x0, y0, x1, y1
    return b


def test_match_recall_equals_oracle_on_random_boxes():
    rng = np.random.default_rng(0)
    for trial in range(200):
        n, m = rng.integers(0, 12), rng.integers(0, 12)

        def rand(k):
            x0 = rng.integers(0, 400, k)
            y0 = rng.integers(0, 200, k)
            w = rng.integers(40, 120, k)
            return [(int(a), int(b), int(a + c), int(b + 2 * c)) for a, b, c in zip(x0, y0, w)]

        a, b = rand(n), rand(m)
        # near-duplicates make the one-to-one matching matter
        b += [(x + int(rng.integers(-8, 9)), y, x1, y1) for x, y, x1, y1 in a[: n // 2]]
        assert T.match_recall(_boxes(a), _boxes(b)) == P.match_recall(a, b), trial
