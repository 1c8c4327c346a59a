"""GPU test of the apply for callers that cannot allocate (hpdg_apply_noalloc): the same result as
hpdg_apply, through the C ABI, on two calls in a row with the second on a smaller mesh, and a
level too large for the fixed scratch is refused with an error."""
import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hp = pytest.importorskip("paper_1907_01572_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = hp.Context(0)
    yield c
    c.close()


def test_apply_noalloc_equals_apply_on_two_calls_second_smaller(ctx):
    meshes = [meshgen.cubed_sphere_shell(level=2, p=4, r_out=1e3), meshgen.hp_sphere_cube(level=2, p_lo=1, p_hi=4, seed=3)]
    for k, m in enumerate(meshes):
        M = ctx.upload(m, build_f32=True)
        print("call", k, "dof", M.n_dof[0], flush=True)
        for dt in (torch.float64, torch.float32):
            g = torch.Generator(device="cuda").manual_seed(10 + k)
            x = torch.randn(M.n_dof[0], dtype=dt, device="cuda", generator=g)
            y_ref = torch.zeros_like(x)
            y = torch.full_like(x, float("nan"))
            M.apply(x, y_ref)
            M.apply_noalloc(x, y)
            torch.cuda.synchronize()
            # the same kernels on the same input: bitwise equal
            assert torch.equal(y, y_ref), (k, dt)
        M.free()


def test_apply_noalloc_refuses_levels_beyond_the_scratch(ctx):
    # 32^3 cells at p = 4: 12 * 25 * 32768 FP64 trace values = 78.6 MB > 64 MiB
    M = ctx.upload(meshgen.unit_cube(5, 4))
    x = torch.ones(M.n_dof[0], dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(hp.HpdgError) as ei:
        M.apply_noalloc(x, y)
    assert ei.value.code == hp.ERR_INVALID_ARG and "bytes of face traces" in str(ei.value)
    M.apply_noalloc(x[: M.n_dof[1]].contiguous(), y[: M.n_dof[1]].contiguous(), level=1)  # a coarser level fits
    M.free()
