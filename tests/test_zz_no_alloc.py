"""grte_mlp_train_noalloc (training that allocates no device memory) against
grte_mlp_train, through the C ABI.

Both run the same kernels in the same order on the same model state and
rows, so parameters, bfloat16 copy and loss history must agree bit for bit.
Two calls in a row: the second with fewer rows and a smaller minibatch, so
the fixed workspace keeps the first call's contents where the second does
not write -- nothing may depend on it.  A request beyond the workspace is
refused and leaves the model unchanged.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1811_05579_amd import GrteError, Mlp
from paper_1811_05579_amd.workloads import mlp_init

pytestmark = pytest.mark.gpu

NORM = np.array([-4.5, -1.0, 2.5, -2.5, -3.0, 2.6, 0.6, 2.0, 1.4, 0.6, 0.0, 0.07], dtype=np.float32)


def _rows(n, seed):
    """Seeded synthetic training rows with the value ranges of logged data."""
    rng = np.random.default_rng(seed)
    F = np.column_stack([rng.uniform(-9, 0, n), rng.uniform(-2, 0, n), rng.uniform(-1, 6, n),
                         rng.uniform(-5, 0, n), rng.uniform(-4, -2, n)])
    t = 0.1 * np.tanh(F[:, 0] + 2 * F[:, 1]) + 0.01 * rng.normal(size=n)
    return np.column_stack([F, t]).astype(np.float32)


def _model():
    m = Mlp()
    m.set_params(mlp_init())
    m.set_norm(NORM)
    return m


def _same(a, b):
    ta, ba = a.get_params()
    tb, bb = b.get_params()
    assert np.array_equal(ta.view(np.uint32), tb.view(np.uint32))
    assert np.array_equal(ba, bb)


def test_noalloc_training_equals_allocating_training():
    ref, new = _model(), _model()
    big = torch.from_numpy(_rows(20000, seed=1)).cuda()
    small = torch.from_numpy(_rows(700, seed=2)).cuda()
    # first call: the largest minibatch the workspace takes (256 blocks), history on
    print("[noalloc] call 1: 20000 rows, batch 16384, 5 steps", flush=True)
    h_ref = ref.train(big, steps=5, batch=16384, lr=1e-3)
    h_new = new.train_noalloc(big, steps=5, batch=16384, lr=1e-3)
    assert np.array_equal(h_ref.view(np.uint32), h_new.view(np.uint32)), (h_ref, h_new)
    _same(ref, new)
    # second call: fewer rows, a ragged minibatch (11 blocks, the last partly
    # filled), more steps than one pass over the rows
    print("[noalloc] call 2: 700 rows, batch 650, 7 steps", flush=True)
    h_ref = ref.train(small, steps=7, batch=650, lr=2e-3)
    h_new = new.train_noalloc(small, steps=7, batch=650, lr=2e-3)
    assert np.array_equal(h_ref.view(np.uint32), h_new.view(np.uint32)), (h_ref, h_new)
    _same(ref, new)
    # without a loss history
    print("[noalloc] call 3: no history", flush=True)
    ref.train(small, steps=2, batch=300, lr=1e-3)
    assert new.train_noalloc(small, steps=2, batch=300, lr=1e-3, history=False) is None
    _same(ref, new)
    ref.close()
    new.close()


def test_noalloc_refuses_requests_beyond_the_workspace():
    m = _model()
    before = m.get_params()[0].copy()
    rows = torch.from_numpy(_rows(20000, seed=3)).cuda()
    with pytest.raises(GrteError):
        m.train_noalloc(rows, steps=1, batch=16385, lr=1e-3)
    with pytest.raises(GrteError):
        m.train_noalloc(rows[:100], steps=65537, batch=64, lr=1e-3)
    assert np.array_equal(m.get_params()[0], before)
    m.close()
