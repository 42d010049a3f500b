"""sfmm_direct_noalloc, the direct sum that allocates nothing (its status word
and partial sums live in the library's fixed per-GPU scratch array), against
sfmm_direct on the same inputs through the C ABI: two calls in a row, the
second with a smaller input, each within 1e-12 relative per target (the same
source chunks give the same summation order, so in practice bit for bit), and
against the CPU oracle's direct sum."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _rel(a, b):
    nb = np.linalg.norm(b, axis=1)
    return (np.linalg.norm(a - b, axis=1) / np.maximum(nb, 1e-6 * np.sqrt((nb ** 2).mean()))).max()


def test_direct_noalloc_matches_direct(orc):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2602_05804_amd as P

    s = P.Solver()
    for n, nt in ((20000, 3000), (5000, 700)):  # the second call is smaller
        print(f"case: direct no-alloc n={n} targets={nt}", flush=True)
        x, m, h = workloads.plummer(n, seed=31 + n)
        xd, md, hd = (torch.from_numpy(a).cuda() for a in (x, m, h))
        tg_h = np.random.default_rng(n).choice(n, nt, replace=False).astype(np.int64)
        tg = torch.from_numpy(tg_h).cuda()
        a0, p0 = s.direct(xd, md, hd, targets=tg)
        acc = torch.empty((nt, 3), dtype=torch.float64, device="cuda")
        pot = torch.empty((nt,), dtype=torch.float64, device="cuda")
        a1, p1 = s.direct(xd, md, hd, targets=tg, no_alloc=True, out=(acc, pot))
        torch.cuda.synchronize()
        a0, p0, a1, p1 = (t.cpu().numpy() for t in (a0, p0, a1, p1))
        assert _rel(a1, a0) <= TOL
        assert (np.abs(p1 - p0) / np.abs(p0)).max() <= TOL
        oa, op = orc.direct(x, m, h, targets=tg_h)
        assert _rel(a1, oa) <= TOL
        assert (np.abs(p1 - op) / np.abs(op)).max() <= TOL
    # every particle as a target
    x, m, h = workloads.polytrope(3000, seed=5)
    xd, md, hd = (torch.from_numpy(a).cuda() for a in (x, m, h))
    a1, p1 = s.direct(xd, md, hd, no_alloc=True)
    a0, p0 = s.direct(xd, md, hd)
    torch.cuda.synchronize()
    assert _rel(a1.cpu().numpy(), a0.cpu().numpy()) <= TOL
    # a target index outside [0, n) is an error, not a read
    with pytest.raises(P.SfmmError, match="out of range"):
        s.direct(xd, md, hd, targets=torch.tensor([3, 3000], device="cuda"), no_alloc=True)
    # more targets than the scratch holds: rejected before any launch
    big = torch.zeros(1_100_000, dtype=torch.int64, device="cuda")
    with pytest.raises(P.SfmmError, match="too many targets"):
        s.direct(xd, md, hd, targets=big, no_alloc=True)
    # the context still works
    a2, _ = s.direct(xd, md, hd, no_alloc=True)
    torch.cuda.synchronize()
    assert np.array_equal(a2.cpu().numpy(), a1.cpu().numpy())
    s.close()
