"""The seeded input generator: determinism, chunking, shapes."""
import numpy as np

from paper_1109_0778_amd import datagen


def test_chunked_equals_one_shot():
    a = datagen.blobs(5000, 6, 5, 5, 1.0, 3, chunk_rows=777)
    b = datagen.blobs(5000, 6, 5, 5, 1.0, 3, chunk_rows=1 << 20)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_deterministic_and_shapes():
    X1, C1 = datagen.workload("small")
    X2, C2 = datagen.workload("small")
    assert X1.dtype == np.float32 and X1.flags.c_contiguous and X1.shape == (4096, 8)
    assert np.array_equal(X1, X2) and np.array_equal(C1, C2)
    assert np.array_equal(C1, X1[:8])          # "first k points" initialisation


def test_sample_init_distinct_rows():
    X, C = datagen.blobs(1000, 4, 50, 10, 1.0, 5)
    rows = {tuple(r) for r in C.tolist()}
    assert len(rows) == 50
    assert all(any(np.array_equal(c, x) for x in X) for c in C[:5])


def test_aniso_sigma_range():
    X, C, ids = datagen.blobs(20000, 3, 4, 4, 1.0, 9, aniso=True, return_ids=True)
    for b in range(4):
        s = X[ids == b].std(0)
        assert np.all(s > 0.4) and np.all(s < 3.3)


def test_batch_shapes():
    shapes = [datagen.batch_instance_shape(i) for i in range(64)]
    assert all(1000 <= s.n <= 200000 and s.d in (16, 32, 64) and 4 <= s.k <= 128 for s in shapes)
    s, X, C = datagen.batch_instance(3)
    assert X.shape == (s.n, s.d) and C.shape == (s.k, s.d)
