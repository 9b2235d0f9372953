"""GPU: elm_gram_noalloc, the Gram step for callers that cannot allocate
device memory, against elm_gram (the same kernels with the partial tiles in
the handle's workspace) through the C ABI.

For each accepted (dtype, layout) the no-allocation entry point is called
twice in a row on one handle, the second time with a smaller input, and each
result must equal elm_gram's on the same input bit for bit: with the default
rule's split count both sum every Gram entry in the same fixed order, and
the second call must not see the first call's partial tiles.  A shape whose
default split count does not fit the static array runs with fewer splits:
its Gram then differs from elm_gram's by FP32 rounding only, and both are
checked against the FP64 Gram of the rounded input under the split-K bound.
Orders beyond the array are rejected before any device work.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

_LP = {"bf16": torch.bfloat16, "fp16": torch.float16, "fp32": torch.float32}


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


def _input(kind, N, L, seed):
    rng = np.random.default_rng(seed)
    H64 = rng.uniform(0, 1, (N, L))
    H64[:, 3 % L] = H64[:, 1 % L]  # a duplicated column
    if kind == "fp64":
        return to_dev(H64), "sample"
    return to_dev(H64.T.copy()).to(_LP[kind]), "node"


@pytest.mark.parametrize("kind,first,second", [
    ("bf16", (20011, 600), (5003, 257)),
    ("fp16", (9000, 530), (3001, 129)),
    ("fp32", (20011, 600), (2000, 200)),
    ("fp64", (20011, 600), (700, 300)),
    ("fp64", (900, 1200), (300, 450)),      # N < L: the H H^T route
])
def test_noalloc_gram_equals_gram_on_two_calls(elm, kind, first, second):
    for call, (N, L) in enumerate((first, second)):
        H, layout = _input(kind, N, L, seed=100 * call + N + L)
        n = min(N, L)
        want = elm.elm_gram(H, layout)
        # the output buffer starts as garbage: every entry must be written
        M = torch.full((n, n), float("nan"), dtype=torch.float64, device=H.device)
        got = elm.elm_gram(H, layout, M=M, noalloc=True)
        torch.cuda.synchronize()
        same = torch.equal(got, want)
        print(f"{kind} call {call + 1}: N={N} L={L}: bitwise equal to elm_gram: {same}")
        assert same


def test_noalloc_gram_with_fewer_splits(elm):
    # L = 2048 (36 upper 256-tiles) over N = 400000 samples: the default rule's
    # 8 splits need 36 x 8 x 256 KiB = 72 MiB of partials, more than the
    # 64 MiB array, so this call runs with 7 splits; elm_gram keeps 8
    N, L = 400000, 2048
    H, layout = _input("bf16", N, L, seed=5)
    want = elm.elm_gram(H, layout)
    got = elm.elm_gram(H, layout, noalloc=True)
    torch.cuda.synchronize()
    Hr = H.double()
    ref = (Hr @ Hr.T).cpu().numpy()   # FP64 Gram of the rounded input
    g, w = got.cpu().numpy(), want.cpu().numpy()
    # FP32 sums over at most ceil(N / splits) samples per work item (rounding
    # grows like sqrt(kc) 2^-24 of the sum), FP64 across items; one split at
    # the least
    bound = 4 * np.sqrt(N) * 2.0 ** -24 * np.max(np.abs(ref))
    print(f"fewer splits: |noalloc - fp64| {np.max(np.abs(g - ref)):.2e}, |elm_gram - fp64| "
          f"{np.max(np.abs(w - ref)):.2e}, bound {bound:.2e}")
    assert np.array_equal(g, g.T)
    assert np.max(np.abs(g - ref)) <= bound
    assert np.array_equal(g[3], g[1])   # duplicated columns: bitwise-equal rows


def test_noalloc_gram_rejects_orders_beyond_the_array(elm):
    # 16-bit Gram of L = 6000 nodes: 276 upper 256-tiles x 256 KiB > 64 MiB
    # even unsplit; the call is refused on the host, nothing is launched
    H = torch.zeros((6000, 8192), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(elm.ElmError) as ei:
        elm.elm_gram(H, "node", noalloc=True)
    assert ei.value.status == 2   # ELM_ERR_SHAPE
