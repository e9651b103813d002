"""The launch-shape autotuner (fr_autotune) on the GPU: it chooses the items
per tile of every stage and degree (degree pair) of the fused plans and the
blocks of the per-bucket launches, and the results of every operator do not
depend on the shapes (each element's and face's arithmetic is the same in any
tile): bitwise equal before and after tuning, in both launch modes."""
import pytest

from paper_1910_03693_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def frx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_03693_amd import frx as F
    F.lib()
    return F


def test_autotuned_shapes_keep_every_result(frx):
    case = I.case_ns_mixed(8, 8, 4, k=63, lengths=(1.0, 1.0, 0.5), pvals=(1, 2, 3, 4, 5), pw=(1, 1, 1, 1, 1),
                           wall=True, re=500.0, ma=0.2)
    ctx = frx.Context.from_case(case, max_restart=0)
    U = torch.tensor(case.U, device="cuda")
    v = torch.tensor(I.random_direction(case.U.size, 4063).reshape(case.U.shape), device="cuda")

    def results():
        out = {}
        for fused in (True, False):
            ctx.set_launch(fused)
            out[(fused, "R")] = ctx.residual(U).clone()
            out[(fused, "Jv")] = ctx.jvp(U, v).clone()
            out[(fused, "J32")] = ctx.jvp(U, v.float(), precision=frx.FR_F32).clone()
            out[(fused, "JTw")] = ctx.vjp(U, v).clone()
        return out

    before = results()
    shapes0 = {k: ctx.launch_shapes(k) for k in range(3)}
    ctx.autotune(U)
    shapes1 = {k: ctx.launch_shapes(k) for k in range(3)}
    after = results()
    print("fused shapes before", shapes0[1], "after", shapes1[1])
    for k in range(3):
        assert [s[:2] for s in shapes0[k]] == [s[:2] for s in shapes1[k]]
        for st, code, items in shapes1[k]:
            threads = code ** 3 if st != 1 else (code % 8) ** 2
            assert 1 <= items and items * threads <= 256
    for key in before:
        assert torch.equal(before[key], after[key]), key
