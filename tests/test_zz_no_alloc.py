"""gp_query_noalloc through the C ABI: the PIP / P2P query with the library's own
workspace equals gp_pip / gp_p2p with a caller workspace bit for bit, on two calls in a
row (the second with fewer points, so the buffer holds the first call's leftovers);
inputs whose workspace exceeds the buffer are refused before any launch."""
import pytest

from paper_1403_0802_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1403_0802_amd import gp as gpmod
    return gpmod


def noalloc(gp, grid, x, y, prec):
    n = x.numel()
    oid = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    od = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = gp.lib.gp_query_noalloc(grid.handle, grid.kind, n, x.data_ptr(), y.data_ptr(),
                                 oid.data_ptr(), od.data_ptr() if grid.kind == gp.GP_P2P else None,
                                 gp.PRECISIONS[prec], stream)
    gp.check(rc)
    torch.cuda.synchronize()
    return oid, od


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("kind", ["pip", "p2p"])
def test_noalloc_equals_workspace_entry_points(gp, kind, prec):
    if kind == "pip":
        w = synth.config1(n_points=50_000)
        sizes = (50_000, 7_001)
    else:
        w = synth.config2(n_points=600_000, n_lines=20_000)
        sizes = (600_000, 123_457)
    print("noalloc", kind, prec, sizes, flush=True)
    grid = gp.gp_build_grid(kind, w.geom, w.params)
    assert gp.gp_workspace_bytes(grid, sizes[0], prec) <= gp.GP_NOALLOC_SCRATCH_BYTES
    x = torch.from_numpy(w.px).cuda()
    y = torch.from_numpy(w.py).cuda()
    for call, n in enumerate(sizes):
        # different points on each call: the second call starts at an offset
        lo = 0 if call == 0 else 1_000
        xs, ys = x[lo:lo + n].contiguous(), y[lo:lo + n].contiguous()
        want = gp.run(grid, xs, ys, prec)
        torch.cuda.synchronize()
        oid, od = noalloc(gp, grid, xs, ys, prec)
        if kind == "pip":
            assert torch.equal(oid, want), f"call {call}: {int((oid != want).sum())} ids differ"
        else:
            assert torch.equal(oid, want[0]), f"call {call}: ids differ"
            assert torch.equal(od, want[1]), f"call {call}: distances differ"
        assert int((oid >= 0).sum()) > 0


def test_noalloc_refuses_inputs_beyond_its_buffer(gp):
    w = synth.config2(n_points=1_000, n_lines=2_000)
    grid = gp.gp_build_grid("p2p", w.geom, w.params)
    n = 1
    while gp.gp_workspace_bytes(grid, n, "mixed") <= gp.GP_NOALLOC_SCRATCH_BYTES:
        n *= 2
    # no point array is touched: the size check comes before any launch
    rc = gp.lib.gp_query_noalloc(grid.handle, gp.GP_P2P, n, None, None, None, None,
                                 gp.GP_MIXED, None)
    assert rc == gp.GP_E_CAPACITY
    assert b"scratch" in gp.lib.gp_last_error()
    assert gp.lib.gp_query_noalloc(None, gp.GP_PIP, 10, None, None, None, None, 0,
                                   None) == gp.GP_E_INVALID_ARG
    assert gp.lib.gp_query_noalloc(grid.handle, 3, 10, None, None, None, None, 0,
                                   None) == gp.GP_E_INVALID_ARG
