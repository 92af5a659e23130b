"""Host logic of the batch autotuner (no GPU): the batch-wide choice is the
fastest candidate, a class keeps its own tiles per block only for a gain of
more than 2%, classes of one instance are not swept, the instances'
centroids are restored, and the cache returns the stored choice without
timing anything."""
import pytest
import torch

from paper_1109_0778_amd import autotune


class FakeBatch:
    """Schedule state and shape classes of a batch; no kernels."""

    precision = "bf16"

    def __init__(self):
        self.instances = [{"X": torch.zeros(n, d), "C": torch.full((k, d), float(i))}
                          for i, (n, d, k) in enumerate([(1000, 16, 4), (2000, 16, 8), (500, 64, 30),
                                                          (800, 64, 20), (300, 32, 5)])]
        self.tpb, self.order = 16, 1
        self.cls = [0, 0, 0]
        self.counts = [2, 2, 1]

    def set_schedule(self, tpb, order):
        self.tpb, self.order = tpb, order

    def set_class_schedule(self, c, v):
        self.cls[c] = v

    def classes(self):
        return [(2 * (c + 1), 24576, self.counts[c], self.cls[c] or self.tpb) for c in range(3)]


def fake_timer(batch):
    """A cost surface with its batch-wide minimum at (8, 0); class 0 gains 5%
    at 32 tiles per block, class 1 only 1% at 2; the 'iteration' moves every
    instance's centroids, which the tuner must undo."""
    for t in batch.instances:
        t["C"] += 1.0
    base = 1.0 + 0.1 * abs({1: 0, 2: 1, 4: 2, 8: 3, 16: 4, 32: 5}[batch.tpb] - 3) + 0.01 * batch.order
    f = 0.95 if batch.cls[0] == 32 else 1.0
    f *= 0.99 if batch.cls[1] == 2 else 1.0
    f *= 1.2 if 64 in batch.cls else 1.0
    return base * f


def test_tuner_choice_and_restore(tmp_path, monkeypatch):
    monkeypatch.setenv("KM_TUNE_CACHE", str(tmp_path / "tune.json"))
    b = FakeBatch()
    C0 = [t["C"].clone() for t in b.instances]
    choice, ms = autotune.tune_batch(b, use_cache=True, timer=fake_timer, arch="test")
    assert choice == (8, 0, [32, 0, 0])
    assert (b.tpb, b.order, b.cls) == (8, 0, [32, 0, 0])
    assert all(torch.equal(t["C"], c) for t, c in zip(b.instances, C0))
    assert len([k for k in ms if "," in k]) == len(autotune.CANDIDATES)
    assert not any(k.startswith("class2:") for k in ms)          # one instance: not swept
    assert "class1:2" in ms and "class0:32" in ms

    def no_timer(_):
        raise AssertionError("a cached choice must not be timed")
    b2 = FakeBatch()
    choice2, _ = autotune.tune_batch(b2, use_cache=True, timer=no_timer, arch="test")
    assert choice2 == (8, 0, [32, 0, 0]) and (b2.tpb, b2.order, b2.cls) == (8, 0, [32, 0, 0])
    # another device or precision is a different cache entry
    with pytest.raises(AssertionError):
        autotune.tune_batch(FakeBatch(), use_cache=True, timer=no_timer, arch="other")


def test_tuner_without_classes():
    b = FakeBatch()
    choice, ms = autotune.tune_batch(b, use_cache=False, per_class=False, timer=fake_timer, arch="test")
    assert choice == (8, 0, [0, 0, 0]) and b.cls == [0, 0, 0]
    assert not any(k.startswith("class") for k in ms)


def test_signature_ignores_small_n_differences():
    a = [{"X": torch.zeros(1000, 16), "C": torch.zeros(4, 16)}]
    b = [{"X": torch.zeros(1004, 16), "C": torch.zeros(4, 16)}]
    c = [{"X": torch.zeros(1000, 32), "C": torch.zeros(4, 32)}]
    assert autotune.signature(a) == autotune.signature(b) != autotune.signature(c)
