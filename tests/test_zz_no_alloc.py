"""pts_eval_noalloc (workspace in the library's static device array) against pts_eval.

Both run the same kernels with the same launch plan, so their results must be
bitwise equal; the first call is also checked against the FP64 oracle at the
evaluator's tolerance.  Two calls in a row, the second on a smaller cloud
with fewer queries, so the second reads the array after a larger call has
left its contents there.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_16946_amd import binding, synth

SCRATCH_BYTES = 64 << 20


def _case(N, Q, seed):
    cl, _ = synth.tiny(Q=16, N=N)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.5, 1.5, size=(Q, 3)).astype(np.float32)
    return cl, x


@pytest.mark.gpu
def test_noalloc_matches_eval_on_two_calls():
    torch.cuda.set_device(0)
    prm = binding.make_params()
    for N, Q, seed, check_oracle in ((20000, 50001, 1, True), (3001, 777, 2, False)):
        print(f"noalloc: N={N} Q={Q}", flush=True)
        cl, x = _case(N, Q, seed)
        assert binding.eval_ws_bytes(N, Q, prm) <= SCRATCH_BYTES
        p, n, a, xd = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a, x))
        rec = binding.cloud_build(p, n, a, prm)
        ref = binding.eval(rec, N, xd, prm)
        got = binding.eval_noalloc(rec, N, xd, prm)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(r.view(np.uint32), g.view(np.uint32)), float(np.abs(r - g).max())
        if check_oracle:
            idx = np.arange(0, Q, 97)
            phi = oracle.sdf(cl.p, cl.n, cl.a, x[idx])
            D = oracle.bbox_diag(cl.p)
            assert np.abs(g[idx].astype(np.float64) - phi).max() <= 1e-5 * D


@pytest.mark.gpu
def test_noalloc_refuses_oversized_plans_and_stays_usable():
    torch.cuda.set_device(0)
    prm = binding.make_params()
    cl, x = _case(4096, 4096, 3)
    p, n, a, xd = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a, x))
    rec = binding.cloud_build(p, n, a, prm)
    Qbig = 1 << 22
    assert binding.eval_ws_bytes(4096, Qbig, prm) > SCRATCH_BYTES
    xbig = torch.zeros((Qbig, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(binding.PtsError, match="static scratch"):
        binding.eval_noalloc(rec, 4096, xbig, prm)
    got = binding.eval_noalloc(rec, 4096, xd, prm)
    ref = binding.eval(rec, 4096, xd, prm)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
