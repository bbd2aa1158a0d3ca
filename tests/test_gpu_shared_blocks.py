"""Patch factors with one A^-1 for every velocity component (share_blocks).

The vector Laplacian with the same boundary conditions on each component
(Section 2) gives every patch identical component blocks, so the library
stores one inverse per patch instead of one per component (Section 3.3.1 keeps
the blocks apart).  The cycle must equal the oracle's with that layout and
with the per-component layout (share_blocks = 0), on bucketed, staged,
full-block and batched levels, FP64 and FP32; a problem whose component blocks
differ (the y-velocity unknowns rescaled) must fall back to per-component
blocks and still equal the oracle's cycle.
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle import dc  # noqa: E402
from paper_2306_06795_amd import mas  # noqa: E402
from parity import assert_parity  # noqa: E402
from test_gpu_parity import build  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHARED = 2  # patch_layout bit of the one-block records


def apply(h, R, nr):
    Rd = torch.tensor(np.ascontiguousarray(R[:, :nr]), device=DEV)
    Zd = torch.empty_like(Rd)
    h.apply(Rd, Zd, nrhs=nr)
    torch.cuda.synchronize()
    return Zd.cpu().numpy().reshape(R.shape[0], nr)


@pytest.mark.parametrize("name,over", [
    ("th24_lid", {}),
    ("th24_lid", {"bucket_min": 1}),    # 19/19 buckets (thread per patch)
    ("sv8_lid", {"bucket_min": 1}),     # 6/6/3-seed buckets
    ("th3d4", {}),
    ("th3d6_3lvl", {"full_patch_min": 100}),  # every 3D level stores full blocks
    ("th3d8_big", {}),                  # coarse records too large for LDS: panels
    ("th16_ho", {}),
])
def test_shared_and_per_component_layouts_match_oracle(name, over):
    P, par, mp = build(name)
    for k, v in over.items():
        setattr(mp, k, v)
    pre = dc.DCPreconditioner(P, par)
    R = np.random.default_rng(29).standard_normal((P.n0, 3))
    refs = [pre.apply(R[:, k]) for k in range(3)]
    mp.nrhs_max = 3
    # (share_blocks, patch_kernel): the workgroup kernel and the persistent
    # pipelined one on both layouts, the shared-block wavefront and panel
    # kernels, the per-component column kernel
    for share, kern in ((1, 1), (1, 3), (1, 4), (1, 5), (0, 1), (0, 2), (0, 4)):
        for precision, tol in ((mas.MAS_FP64, 1e-11), (mas.MAS_FP32, 1e-5)):
            mp.share_blocks, mp.patch_kernel, mp.precision = share, kern, precision
            h = mas.Handle(P, mp)
            info = h.info()
            relaxed = [l for l in range(info["n_levels"]) if info["n_patches"][l] > 0]
            print(f"[{name} {over}] share {share} kernel {kern} precision {precision}: layouts "
                  f"{info['patch_layout']} kernels {info['patch_kernel']}", flush=True)
            assert relaxed and all(bool(info["patch_layout"][l] & SHARED) == bool(share) for l in relaxed)
            assert all(info["patch_kernel"][l] in (0, 1, kern) for l in relaxed)
            if kern in (2, 3, 5) and (share or kern == 2) and "full_patch_min" not in over:
                # packed blocks: the kernel applies somewhere
                assert any(info["patch_kernel"][l] == kern for l in relaxed)
            for nr in (1, 3):
                Z = apply(h, R, nr)
                for k in range(nr):
                    assert_parity(Z[:, k], refs[k], P.field0, tol,
                                  f"share {share} kernel {kern} prec {precision} nr {nr} col {k}")
            h.close()


def rescaled(P, s=2.0):
    """The free y-velocity unknowns of K0 and K1 scaled by s (D K D): the
    component-1 blocks become s^2 times the component-0 blocks."""
    def scale(K, field, dirichlet):
        d = np.where((field == 1) & ~dirichlet, s, 1.0)
        D = sp.diags(d)
        return (D @ K @ D).tocsr()
    return dataclasses.replace(P, K0=scale(P.K0, P.field0, P.dir0), K1=scale(P.K1, P.field1, P.dir1))


@pytest.mark.parametrize("name", ["th24_lid", "th3d4"])
def test_distinct_component_blocks_keep_one_block_each(name):
    P0, par, mp = build(name)
    P = rescaled(P0)
    pre = dc.DCPreconditioner(P, par)
    r = np.random.default_rng(31).standard_normal(P.n0)
    ref = pre.apply(r)
    h = mas.Handle(P, mp)
    info = h.info()
    print(f"[{name} rescaled] layouts {info['patch_layout']}", flush=True)
    assert not any(info["patch_layout"][l] & SHARED for l in range(info["n_levels"]))
    Z = apply(h, r[:, None], 1)
    assert_parity(Z[:, 0], ref, P.field0, 1e-11, "rescaled y-velocity")
    h.close()
