"""The allocation-free prediction entry point against the one that takes a
workspace argument: same kernels, same chunking, so the outputs agree bit for
bit; two calls in a row on one device, the second on a smaller grid, for the
per-state and the level form."""
import numpy as np
import pytest

from paper_2103_00331_amd import instances as I
from tests.parity import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    from paper_2103_00331_amd import binding
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return binding


@pytest.mark.parametrize("level", [False, True])
@pytest.mark.parametrize("precision", [1, 2])
def test_noalloc_predict_matches_workspace_predict(B, level, precision):
    params = torch.empty(B.cpmdp_mlp_param_count(), dtype=torch.float32, device="cuda")
    B.cpmdp_mlp_init(params, 5)
    params += 0.05 * torch.randn(params.numel(), device="cuda",
                                 generator=torch.Generator("cuda").manual_seed(6))
    for m, chunk in ((20, 4096), (9, 300)):           # the second call on a smaller grid
        x = I.warm_instance(2, 3, m=m)
        log(f"[noalloc] m={m} chunk={chunk} level={level} precision={precision}")
        R = torch.as_tensor(x.rewards, dtype=torch.float32, device="cuda")
        ref = torch.full((x.n_states,), np.nan, dtype=torch.float64, device="cuda")
        got = torch.full_like(ref, np.nan)
        ws = torch.empty(B.cpmdp_mlp_workspace_bytes(chunk), dtype=torch.uint8, device="cuda")
        B.cpmdp_mlp_predict(params, R, m, x.gamma, x.meta["slip"], ref, chunk, ws,
                            precision=precision, level=level)
        B.cpmdp_mlp_predict_noalloc(params, R, m, x.gamma, x.meta["slip"], got, chunk,
                                    precision=precision, level=level)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(got).all())
        assert torch.equal(got, ref)


def test_noalloc_rejects_chunk_above_scratch(B):
    x = I.warm_instance(2, 3, m=9)
    params = torch.zeros(B.cpmdp_mlp_param_count(), dtype=torch.float32, device="cuda")
    R = torch.as_tensor(x.rewards, dtype=torch.float32, device="cuda")
    V = torch.zeros(x.n_states, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CpmdpError) as e:
        B.cpmdp_mlp_predict_noalloc(params, R, 9, x.gamma, x.meta["slip"], V, 4097)
    assert e.value.code == B.CPMDP_E_ARG
