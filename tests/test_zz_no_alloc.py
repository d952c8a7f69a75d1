"""GPU test of cfr_mlp_forward_noalloc, the inference entry point that allocates nothing (its hidden
activations live in the library's static device scratch): through the C ABI, its logits equal those of
cfr_mlp_forward bitwise, on two calls in a row (the second with fewer rows, over the scratch the first
left behind), and more rows than the scratch holds are refused."""
import numpy as np
import pytest

import gamegen as gg
import paper_2609_11923_amd as cfr

pytestmark = pytest.mark.gpu


def test_noalloc_forward_equals_forward_on_two_calls():
    torch = pytest.importorskip("torch")
    net = cfr.Mlp(max_rows=4096)
    sizes = [(cfr.CFR_FEATURES, 256), (256, 256), (256, 256), (256, cfr.CFR_MLP_OUT)]
    net.set_params(gg.mlp_init(sizes, seed=11))
    rng = np.random.default_rng(3)
    for rows in (8192, 1000):
        x = torch.tensor(rng.standard_normal((rows, cfr.CFR_FEATURES)), dtype=torch.bfloat16, device="cuda")
        za = torch.full((rows, 4), np.nan, dtype=torch.float32, device="cuda")
        zb = torch.full((rows, 4), np.nan, dtype=torch.float32, device="cuda")
        net.forward(x, rows, za)
        net.forward_noalloc(x, rows, zb)
        torch.cuda.synchronize()
        a, b = za.cpu().numpy(), zb.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), rows


def test_noalloc_forward_refuses_more_rows_than_the_scratch():
    torch = pytest.importorskip("torch")
    net = cfr.Mlp()
    x = torch.zeros((8193, cfr.CFR_FEATURES), dtype=torch.bfloat16, device="cuda")
    z = torch.empty((8193, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(cfr.CfrError) as e:
        net.forward_noalloc(x, 8193, z)
    assert e.value.status == cfr.CFR_EINVAL and "8192" in str(e.value)
    net.forward_noalloc(x, 0, z)   # an empty call is a no-op
