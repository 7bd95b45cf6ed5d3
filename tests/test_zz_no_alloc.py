"""mvpf_residual_noalloc (the entry point for callers that cannot allocate
device memory) against mvpf_residual through the C ABI: same residual and
free-dof norm, bitwise (the same kernels; slab boundaries do not change the
arithmetic), on two calls in a row, the second on a smaller problem, plus the
size limit of its fixed scratch."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import gpu_problem, say, seeded_state

pytestmark = pytest.mark.gpu


def _compare(p, u_amp, depth, tag):
    from paper_2011_08802_amd import mvpf
    U, En = seeded_state(p, u_amp, seed=31)
    say(f"[no-alloc {tag}] {p.nx}x{p.ny}x{p.nz}, {p.n_levels} levels")
    gp = gpu_problem(p, U, En, "mixed", depth=depth)
    R0, n0 = gp.residual()
    # a caller-owned output filled with garbage first: every entry is written
    R1 = torch.full_like(R0, float("nan"))
    R1, n1 = gp.residual_noalloc(R1)
    gp.close()
    assert torch.equal(R0, R1), float((R0 - R1).abs().max())
    assert n0 == n1 and np.isfinite(n0) and n0 > 0, (n0, n1)
    return R0


def test_noalloc_residual_matches_residual():
    from paper_2011_08802_amd import mvpf
    lim = mvpf.load().mvpf_residual_noalloc_max_layer()
    # 48^3 elements: 48 * 48 = 2304 per layer, 110592 in all, more than one
    # slab of the fixed scratch holds, so several slabs run
    big = synth.Problem(48, 48, 48, n_levels=4, patch=6, depth_increment=0.01)
    assert 48 * 48 <= lim and 48 ** 3 > 2 * lim
    _compare(big, 2e-3, 0.01, "two slabs")
    small = synth.Problem(16, 16, 8, lz=0.5, n_levels=2, patch=4, depth_increment=0.01)
    _compare(small, 1e-3, 0.005, "smaller")


def test_noalloc_residual_contact():
    """Sphere-contact loading: the contact term is part of both residuals."""
    p = synth.Problem(16, 16, 8, lz=0.5, n_levels=2, kind="sphere", radius=0.5, eps_n=3.5e4,
                      depth_increment=0.01)
    _compare(p, 0.0, 0.02, "contact")


def test_noalloc_rejects_wide_layers():
    from paper_2011_08802_amd import mvpf
    lim = mvpf.load().mvpf_residual_noalloc_max_layer()
    p = synth.Problem(192, 192, 16, lz=16 / 192, n_levels=5, patch=8, depth_increment=0.01)
    assert 192 * 192 > lim
    say(f"[no-alloc limit] 192x192x16 (limit {lim} elements per layer)")
    gp = mvpf.Problem(p, "mixed")
    with pytest.raises(mvpf.MvpfError, match="exceeds the fixed scratch"):
        gp.residual_noalloc()
    gp.close()
