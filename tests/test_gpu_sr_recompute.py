"""SR with O recomputed from the spins in chunks (for batches whose O does not
fit in device memory).  Chunks are whole reduction blocks of the solve, so the
result must equal the stored-O solve on log_deriv's O bit for bit, for every
chunk size; and the stored-O solve is itself checked against the oracle's CG
in test_gpu_grad_sr.py.  Here the recompute variant is also checked against
the oracle's CG directly on one case."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07816_amd import inputs
from gpu_helpers import DEV, make_ctx, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    # name, L, J2, K, C, B, sigma, O dtype, chunk_rows list, dtype of the context
    ("10x10 K4 C16 B=300 fp64", 10, 0.5, 4, 16, 300, 0.1, "fp64", [0, 1, 60, 61, 299], "fp64"),
    ("10x10 K4 C16 B=300 fp32", 10, 0.5, 4, 16, 300, 0.1, "fp32", [60, 150], "fp64"),
    ("24x24 K6 C32 B=192 fp32 bf16 ctx", 24, 0.5, 6, 32, 192, 0.05, "fp32", [64, 100], "bf16"),
]


@pytest.mark.parametrize("name,L,J2,K,C,B,sigma,odt,chunks,cdt", CASES,
                         ids=[c[0] for c in CASES])
def test_recompute_equals_stored(name, L, J2, K, C, B, sigma, odt, chunks, cdt):
    say("case", name)
    w = inputs.weights(K, C, sigma, 21)
    sp = to_dev(inputs.spins_sz0(L, B, 22))
    ctx = make_ctx(L, J2, K, C, w, dtype=cdt)
    e = ctx.local_energy(sp, mode="full")
    O = ctx.log_deriv(sp, dtype=odt)
    x_ref, st_ref = ctx.sr_solve(O, e, 1e-4, 30)
    x_ref, st_ref = x_ref.clone(), st_ref.clone()
    del O
    for ch in chunks:
        x, st = ctx.sr_solve_recompute(sp, e, 1e-4, 30, dtype=odt, chunk_rows=ch)
        torch.cuda.synchronize()
        say("  chunk_rows", ch, "max |dx|", float((x - x_ref).abs().max()))
        assert torch.equal(x, x_ref), f"chunk_rows={ch}"
        assert torch.equal(st, st_ref), f"chunk_rows={ch}"
    assert ctx.get_error() == 0


def test_recompute_vs_oracle_cg():
    L, K, C, B = 4, 2, 4, 256
    w = inputs.weights(K, C, 0.1, 13)
    sp = inputs.spins_sz0(L, B, 14)
    O = oracle.log_deriv(L, K, C, w, sp)
    e = oracle.local_energy(L, 1.0, 0.5, K, C, w, sp)
    ctx = make_ctx(L, 0.5, K, C, w)
    x, st = ctx.sr_solve_recompute(to_dev(sp), torch.tensor(e, device=DEV), 1e-4, 100,
                                   dtype="fp64", chunk_rows=40)
    ref, rel, it = oracle.sr_cg(O, e, 1e-4, 100)
    x = x.cpu().numpy()
    say("  |dx|/|x|", np.linalg.norm(x - ref) / np.linalg.norm(ref))
    assert np.linalg.norm(x - ref) <= 1e-6 * np.linalg.norm(ref)


def test_recompute_argument_errors():
    L, K, C, B = 4, 2, 4, 16
    ctx = make_ctx(L, 0.5, K, C, inputs.weights(K, C, 0.1, 1))
    sp = to_dev(inputs.spins_sz0(L, B, 2))
    e = torch.zeros(B, dtype=torch.float64, device=DEV)
    with pytest.raises(Exception):
        ctx.sr_solve_recompute(sp, e, 1e-4, 10, chunk_rows=-1)
    with pytest.raises(Exception):
        ctx.sr_solve_recompute(sp, e, -1.0, 10)
    x, st = ctx.sr_solve_recompute(sp, e, 1e-4, 10)   # E constant: F = 0
    assert torch.all(x == 0) and st[3].item() == 0
