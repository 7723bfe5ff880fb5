"""The persistent kernels' bounded grid-barrier wait, forced from the host:
with a zero wait limit (BC_BARRIER_TIMEOUT_MS=0, read when a context is
created) every workgroup that would wait gives up, raises the abort word and
returns, so the launch ends normally and the call reports BC_E_DEVICE.  A
context with the default limit then computes correct scores on the same
device."""
import os
import sys

import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_barrier_give_up_is_reported_and_harmless(mode):
    import paper_1602_00963_amd as bcm
    from paper_1602_00963_amd import bc as bcmod
    g = gg.rmat(10, 8, 77)
    S = gg.sample(g.non_isolated(), 96, 2)
    say("case barrier give-up", mode)
    os.environ["BC_BARRIER_TIMEOUT_MS"] = "0"
    try:
        ctx0 = bcm.Context(0)
    finally:
        del os.environ["BC_BARRIER_TIMEOUT_MS"]
    G0 = bcm.Graph(ctx0, g)
    with pytest.raises(bcm.BCError) as e:
        G0.compute(S, mode=mode, batch=64)
    assert e.value.status == bcmod.E_DEVICE
    assert "barrier" in str(e.value)
    G0.close()
    ctx0.close()
    ctx = bcm.Context(0)
    G = bcm.Graph(ctx, g)
    G.compute(S, mode=mode, batch=64)
    ref, _ = oracle.bc(g, S)
    assert oracle.close(G.scores(), ref, 1e-9).all()
    G.close()
    ctx.close()
