"""The no-allocation variant of decode + query (gsff_decoder_query_noalloc,
scratch in a fixed per-GPU device array) against the workspace entry point
gsff_decoder_query, through the C ABI: identical probabilities, labels and
cross-entropy on two calls in a row, the second with fewer pixels and
labels, and again on the first input (the shared scratch is reused)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _case(rng, n, K):
    X = torch.from_numpy(rng.normal(size=(16, n)).astype(np.float32)).to(torch.bfloat16).cuda()
    W1 = torch.from_numpy((rng.normal(size=(16, 128)) / 4).astype(np.float32)).cuda()
    b1 = torch.from_numpy((rng.normal(size=128) * 0.1).astype(np.float32)).cuda()
    W2 = torch.from_numpy((rng.normal(size=(128, 512)) / 11).astype(np.float32)).cuda()
    b2 = torch.from_numpy((rng.normal(size=512) * 0.1).astype(np.float32)).cuda()
    Q = torch.from_numpy((rng.normal(size=(K, 512)) / 22).astype(np.float32)).cuda()
    gt = torch.from_numpy(rng.integers(-1, K + 1, size=n).astype(np.int32)).cuda()
    return X, W1, b1, W2, b2, Q, gt


def _run(L, args, K, n, noalloc):
    X, W1, b1, W2, b2, Q, gt = args
    prob = torch.full((K, n), -1.0, device="cuda")
    label = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    loss = torch.full((1,), -1.0, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    head = [_p(X), _p(W1), _p(b1), _p(W2), _p(b2), _p(Q), K, n, _p(prob), _p(label), _p(gt),
            _p(loss)]
    if noalloc:
        rc = L.gsff_decoder_query_noalloc(*head, s)
    else:
        nb = ctypes.c_size_t(0)
        assert L.gsff_decoder_query_workspace_size(K, n, ctypes.byref(nb)) == 0
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
        rc = L.gsff_decoder_query(*head, _p(ws), ws.numel(), s)
    assert rc == 0
    torch.cuda.synchronize()
    return prob.cpu().numpy(), label.cpu().numpy(), float(loss.item())


def test_noalloc_query_matches_workspace_entry_point():
    from paper_2504_19409_amd import _capi
    L = _capi.load()
    rng = np.random.default_rng(2024)
    big = (70_001, 37)   # ragged pixel count, three label tiles
    small = (1_003, 5)   # fewer pixels and labels
    a = _case(rng, big[0], big[1])
    b = _case(rng, small[0], small[1])
    for args, (n, K) in [(a, big), (b, small), (a, big)]:
        print(f"case n={n} K={K}", flush=True)
        ref = _run(L, args, K, n, noalloc=False)
        got = _run(L, args, K, n, noalloc=True)
        np.testing.assert_array_equal(got[1], ref[1])  # labels: bit-exact
        np.testing.assert_array_equal(got[0], ref[0])  # same kernels, same arithmetic
        assert got[2] == ref[2]
        assert np.all(got[1] >= 0) and np.all(got[1] < K)
        np.testing.assert_allclose(got[0].sum(axis=0), 1.0, rtol=1e-5)
