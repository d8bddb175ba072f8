"""The seeded generators are deterministic and produce the shapes they promise."""
import json
import os

import numpy as np

from paper_1406_5161_amd import datagen as g

HERE = os.path.dirname(os.path.abspath(__file__))


def test_generator_hashes_are_stable():
    from tests.golden.make_golden import hashes
    want = json.load(open(os.path.join(HERE, "golden", "datagen_sha256.json")))
    got = json.loads(json.dumps(hashes()))
    assert got == want


def test_csr_structure_and_statistics():
    c = g.config2(n=5000)
    d = c.data
    L = np.diff(d.row_ptr)
    assert d.row_ptr[0] == 0 and np.all(L >= 1)
    for i in range(0, d.n, 97):
        cols = d.col[d.row_ptr[i]:d.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and cols.min() >= 0 and cols.max() < d.d
    assert abs(L.mean() - 0.12 * 300) < 1.0
    assert np.all(d.val == 1.0)
    assert abs((d.y > 0).mean() - 0.5) < 0.03


def test_text_like_rows_are_unit_norm():
    d = g.gen_text_like(500, 4000, 75.0, g.rng_for(3, 7))
    sq = np.add.reduceat(d.val.astype(np.float64) ** 2, d.row_ptr[:-1])
    np.testing.assert_allclose(sq, 1.0, atol=1e-6)
    assert abs(np.diff(d.row_ptr).mean() - 75) < 3


def test_serving_stream_shape():
    reqs = g.config5(num=40)
    arr = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(arr) >= 0) and arr[0] == 0.0
    assert all(1000 <= r.config.data.n <= 50000 for r in reqs)
    assert {r.config.data.d for r in reqs} <= {20, 128, 300}
