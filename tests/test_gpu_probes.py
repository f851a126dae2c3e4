"""The two measurement probes behind design decisions of the stage kernel,
checked for what they compute (their timings are taken by bench.py):

* ssd_probe_contraction: `reps` explicit steps x <- x - 0.01 D (I x)^2
  along every line of every cell (Burgers' equation with the N = 4
  flux-point operators of Sec. 3.1), vector-ALU and MFMA variants, against
  the same steps in FP64 with the oracle's operator tables;
* ssd_probe_stream: c = 0.75 a + 0.25 b in all three access variants, and
  its argument checks.
"""
import numpy as np
import pytest

from oracle.basis import Operators

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def handle(torch_cuda):
    from paper_1503_02198_amd import Mesh
    from workloads import cases as C
    from workloads import meshes as M
    return Mesh(M.box_mesh(2, 2), C.vortex_case(), 4, device=0)


def test_contraction_probe(torch_cuda, handle):
    torch = torch_cuda
    cells, reps = 192, 3
    print("case: contraction probe, cells", cells, "reps", reps, flush=True)
    rng = np.random.default_rng(11)
    q = (1.0 + 0.1 * rng.random((4, 4, 4, cells))).astype(np.float32)
    ops = Operators(4)
    x = q.astype(np.float64)
    for _ in range(reps):
        a = np.einsum("ki,vwic->vwkc", ops.I, x)
        x = x - 0.01 * np.einsum("ik,vwkc->vwic", ops.D, a * a)
    scale = np.abs(x).max()
    qd = torch.from_numpy(q.ravel()).to("cuda:0")
    for variant in (0, 1):
        out = torch.empty_like(qd)
        handle.probe_contraction(variant, cells, reps, qd, out)
        got = out.cpu().numpy().reshape(4, 4, 4, cells).astype(np.float64)
        err = np.abs(got - x).max() / scale
        print("variant", variant, "max error relative to the largest value", err)
        assert err < 1e-5
        # the steps moved the state by far more than the tolerance
        assert np.abs(x - q).max() / scale > 1e-3


def test_stream_probe(torch_cuda, handle):
    torch = torch_cuda
    n = 5 * 1024
    print("case: stream probe, n", n, flush=True)
    g = torch.Generator().manual_seed(5)
    a = torch.rand(n, generator=g).to("cuda:0")
    b = torch.rand(n, generator=g).to("cuda:0")
    ref = (0.75 * a.double() + 0.25 * b.double())
    for variant in (0, 1, 2):
        c = torch.full_like(a, float("nan"))
        handle.probe_stream(variant, n, a, b, c)
        err = float((c.double() - ref).abs().max().item())
        print("variant", variant, "max abs error", err)
        assert err <= 2.0 ** -23   # values below 1: within one rounding of the exact result
    c = torch.empty(1000, device="cuda:0")
    with pytest.raises(Exception):
        handle.probe_stream(0, 1000, a[:1000], b[:1000], c)   # not a multiple of 1024
    c = torch.empty(n, device="cuda:0")
    with pytest.raises(Exception):
        handle.probe_stream(3, n, a, b, c)                    # no such variant
