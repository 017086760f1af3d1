"""The batched path's Z = D^T Theta block shapes and their autotuner: every shape gives the
same solve bit for bit (each 32 x 32 output tile is accumulated by the same instruction
sequence), the tuner picks an eligible one, and its choice is kept in the cache file."""
import os

import numpy as np
import pytest

from paper_1412_4080_amd import datagen
from tests._util import dev_matrix

pytestmark = pytest.mark.gpu

NSHAPE = 7


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def _batch(N, K, nsig, seed):
    import torch
    D = datagen.gaussian_dictionary(N, K, seed)
    ys = [datagen.to_storage(datagen.lasso_signal(D, 300 + j)[0], "f32") for j in range(nsig)]
    Y = torch.from_numpy(np.stack(ys).astype(np.float32)).cuda().T
    return dev_matrix(D, "bf16"), Y, datagen.lambda_ratios(nsig, 0.1, 0.9, seed)


def _solve(B, Dd, Y, ratios, L, shape=None):
    if shape is None:
        os.environ.pop("DS_BATCH_TILE", None)
    else:
        os.environ["DS_BATCH_TILE"] = str(shape)
    try:
        X, infos, mask = B.solve(Dd, Y, ratios, step_L=L, gap_tol=1e-6, max_iter=20000,
                                 screened=True)
    finally:
        os.environ.pop("DS_BATCH_TILE", None)
    return X.cpu().numpy(), infos, mask.cpu().numpy()


def test_every_block_shape_gives_the_same_solve(B):
    # K = 1500 pads to 1536 atoms (a multiple of 256) and 128 signals fill two 64-signal
    # blocks, so every shape is eligible
    Dd, Y, ratios = _batch(320, 1500, 128, 3)
    L = B.spectral_norm_sq(Dd, 300)
    X0, i0, m0 = _solve(B, Dd, Y, ratios, L, 0)
    assert all(i["status"] == 0 for i in i0)
    for k in range(1, NSHAPE):
        X, infos, mask = _solve(B, Dd, Y, ratios, L, k)
        assert B.batch_shape()[0] == k
        assert np.array_equal(X, X0), k
        assert np.array_equal(mask, m0), k
        assert [i["iters"] for i in infos] == [i["iters"] for i in i0], k
        assert [i["gap"] for i in infos] == [i["gap"] for i in i0], k


def test_autotuner_choice_and_cache_file(B, tmp_path):
    cache = tmp_path / "tune.txt"
    os.environ["DS_AUTOTUNE_CACHE"] = str(cache)
    try:
        Dd, Y, ratios = _batch(300, 1300, 96, 4)   # a shape not tuned before in this process
        L = B.spectral_norm_sq(Dd, 300)
        X, infos, _ = _solve(B, Dd, Y, ratios, L)
        k, ta, ts = B.batch_shape()
        assert 0 <= k < NSHAPE and ta >= 32 and ts >= 32
        # the padded sizes the chosen block must tile: K to a multiple of 128, B of 64
        assert 1408 % ta == 0 and 128 % ts == 0
        lines = cache.read_text().split()
        assert lines[:4] == ["300", "1300", "96", "bf16"] and int(lines[4]) == k
        X0, i0, _ = _solve(B, Dd, Y, ratios, L, 0)
        assert np.array_equal(X, X0)
        assert [i["iters"] for i in infos] == [i["iters"] for i in i0]
    finally:
        os.environ.pop("DS_AUTOTUNE_CACHE", None)
