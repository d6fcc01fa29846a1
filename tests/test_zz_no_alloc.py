"""fcsph_spectral_lap_noalloc (the entry point for callers that cannot
allocate) against fcsph_spectral_lap through the C ABI: the same kernels in
the same order, so the outputs agree bitwise; two calls in a row on one GPU,
the second on a smaller lattice, each checked; a lattice beyond the static
scratch is refused with a clear error."""
import numpy as np
import pytest

from gpu_helpers import problem, spec, to_dev
from paper_2606_06247_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_06247_amd import api
    assert torch.cuda.is_available()
    return api.Context(0)


SEQS = [
    # (first lattice, second smaller lattice, precision, op_eval)
    (spec((1024, 1024), (True, True)), spec((64, 64), (True, True)), "fp64", "fft_window"),
    (spec((200, 181), (True, True), vel=(("D", "N"), ("N", "D"))), spec((48, 37), (False, True)), "fp64", "fft"),
    (spec((96, 80), (True, True)), spec((33, 40), (True, True)), "fp32", "fft_window"),
    (spec((128, 96), (True, True)), spec((40, 33), (True, False), vel=(("N", "D"), None)), "fp64", "direct"),
    (spec((64, 72, 48), (False, True, False)), spec((24, 33, 16), (False, True, False)), "fp64", "fft_window"),
]


@pytest.mark.parametrize("first,second,precision,op_eval", SEQS,
                         ids=[f"{a['n']}-then-{b['n']}-{p}-{o}" for a, b, p, o in SEQS])
def test_noalloc_lap_equals_lap(ctx, first, second, precision, op_eval):
    import torch
    from paper_2606_06247_amd import api
    for k, s in enumerate((first, second)):
        plan = api.Plan(ctx, problem(s, precision=precision, op_eval=op_eval))
        shape = tuple(reversed(s["n"]))
        for fc in (api.VELOCITY, api.PRESSURE):
            f = to_dev(synth.random_field(shape, 70 + 2 * k + fc))
            ref = plan.spectral_lap(f, fc)
            got = plan.spectral_lap_noalloc(f, fc)
            torch.cuda.synchronize()
            print(f"call {k} {s['n']} {precision} {op_eval} field {fc}: max |diff| "
                  f"{float((got - ref).abs().max()):.3e}", flush=True)
            assert torch.equal(got, ref), (k, s["n"], fc)


def test_noalloc_lap_refuses_beyond_the_scratch(ctx):
    import torch
    from paper_2606_06247_amd import api
    s = spec((160, 160, 160), (False, True, False))
    plan = api.Plan(ctx, problem(s))
    f = torch.zeros((160, 160, 160), dtype=torch.float64, device="cuda")
    with pytest.raises(api.FcsphError, match="static scratch"):
        plan.spectral_lap_noalloc(f)
    # the plan itself still works, and so does the call on a fitting lattice
    plan.spectral_lap(f)
    small = api.Plan(ctx, problem(spec((24, 33, 16), (False, True, False))))
    g = to_dev(np.ones((16, 33, 24)))
    assert torch.equal(small.spectral_lap_noalloc(g), small.spectral_lap(g))
