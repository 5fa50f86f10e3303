"""Batching form of the forcing loop: graph capture and replay
(ibmx_forcing_graph) and the tile-shape autotuner (ibmx_tune), checked
against eager calls and the oracle."""
import numpy as np
import pytest

from paper_2109_03972_amd import synth
from _util import dev_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _setup(case, precision):
    from paper_2109_03972_amd import ibmx
    D = dev_case(case, precision)
    plan = ibmx.Plan.from_case(case, precision)
    plan.set_markers(D["body"], D["dV"])
    return plan, D


def _mask(case, dev):
    import oracle
    import torch
    m = oracle.marker_mask(case, oracle.pairs(case))
    return m, torch.as_tensor(m).to(dev)


def _run(plan, D, u0, mk, graph, resid=None):
    import torch
    D["u"].copy_(u0)
    D["f"].zero_()
    S, T = plan.forcing(D["u"], D["f"], D["xp"], D["up"], D["wp"], mask=mk, resid=resid,
                        graph=graph)
    plan.check("graph" if graph else "eager")
    torch.cuda.synchronize()
    out = dict(u=D["u"].double().cpu().numpy(), f_tot=D["f"].double().cpu().numpy(),
               S=S.cpu().numpy(), T=T.cpu().numpy())
    if resid is not None:
        out["resid"] = resid.cpu().numpy().copy()
    return out


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_graph_replays_match_eager_and_oracle(oracle_lib, precision):
    import torch
    dev = require_gpu()
    case = synth.small_case(71, n=(40, 36, 44), periodic=(1, 1, 0), n_iter=3, touch=0.4)
    m_np, mk = _mask(case, dev)
    plan, D = _setup(case, precision)
    u0 = D["u"].clone()
    resid = torch.zeros(int(case.params["n_iter"]) + 1, dtype=torch.float64, device=dev)
    eager = _run(plan, D, u0, mk, False, resid)
    ref = oracle_lib.forcing(case, mask=m_np)
    tol = 1e-12 if precision == "f64" else 1e-4
    for rep in range(4):
        resid.fill_(-1.0)
        got = _run(plan, D, u0, mk, True, resid)
        # eager torch work between replays
        _ = (D["u"] * 2.0).sum().item()
        for k in ("u", "f_tot", "S", "T", "resid"):
            e = rel_err(got[k], ref[k])
            assert e <= tol, f"replay {rep} {k}: {e:.3e}"
            # integer fixed-point spreading, per-tile residual partials added
            # in tile order, particle sums in marker order: replays are
            # bit-identical to the eager call in both precisions
            np.testing.assert_array_equal(got[k], eager[k], err_msg=f"replay {rep} {k}")


def test_graph_recaptures_on_new_pointers_and_params(oracle_lib):
    import torch
    dev = require_gpu()
    case = synth.small_case(72, n=(38, 40, 42), periodic=(1, 1, 0), n_iter=2, touch=0.4)
    m_np, mk = _mask(case, dev)
    plan, D = _setup(case, "f64")
    u0 = D["u"].clone()
    got = _run(plan, D, u0, mk, True)
    ref = oracle_lib.forcing(case, mask=m_np)
    assert rel_err(got["u"], ref["u"]) <= 1e-12
    # other output buffers: a new capture
    D2 = dict(D)
    D2["u"] = torch.empty_like(D["u"])
    D2["f"] = torch.empty_like(D["f"])
    got2 = _run(plan, D2, u0, mk, True)
    for k in ("u", "f_tot", "S", "T"):
        assert rel_err(got2[k], ref[k]) <= 1e-12, k
    # fewer passes: the captured graph is dropped with the old parameters
    prm = dict(case.params)
    prm["n_iter"] = 1
    plan.set_params(prm)
    got3 = _run(plan, D2, u0, mk, True)
    ref3 = oracle_lib.forcing(case, mask=m_np, n_iter=1)
    for k in ("u", "f_tot", "S", "T"):
        assert rel_err(got3[k], ref3[k]) <= 1e-12, k


def test_switching_delta_kernel_on_a_plan(oracle_lib):
    """ibmx_plan_set_params from the three- to the four-point delta and back
    on one plan (eager and graph calls; the captured graph is dropped with
    the old parameters): each call matches the oracle with that kernel."""
    dev = require_gpu()
    case = synth.small_case(77, n=(40, 36, 44), periodic=(1, 1, 0), n_iter=2, touch=0.4)
    p3 = dict(case.params)
    p4 = dict(p3, kernel=4, eps_sep=2.0, lub_C=4.0, gap_cut=4.0)
    m_np, mk = _mask(case, dev)          # the wider mask of the four-point parameters
    case.params = p4
    m4, mk4 = _mask(case, dev)
    case.params = p3
    plan, D = _setup(case, "f64")
    u0 = D["u"].clone()
    for prm, mask_np, mask_dev in ((p3, m_np, mk), (p4, m4, mk4), (p3, m_np, mk)):
        plan.set_params(prm)
        case.params = prm
        ref = oracle_lib.forcing(case, mask=mask_np)
        for graph in (False, True):
            got = _run(plan, D, u0, mask_dev, graph)
            for k in ("u", "f_tot", "S", "T"):
                e = rel_err(got[k], ref[k])
                assert e <= 1e-12, f"kernel {prm['kernel']} graph {graph} {k}: {e:.3e}"
    case.params = p3


def test_new_marker_offsets_drop_the_graph(oracle_lib):
    """Markers turn with their particle between steps: new body offsets set
    on a plan whose call was captured must be the ones the next graph call
    uses."""
    import torch
    dev = require_gpu()
    case = synth.small_case(78, n=(40, 36, 44), periodic=(1, 1, 0), n_iter=2, touch=0.4)
    m_np, mk = _mask(case, dev)
    plan, D = _setup(case, "f64")
    u0 = D["u"].clone()
    _run(plan, D, u0, mk, True)
    th = 0.3
    rot = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    body2 = rot @ case.body
    plan.set_markers(torch.as_tensor(body2).to(dev).contiguous(), D["dV"])
    got = _run(plan, D, u0, mk, True)
    case2 = synth.Case(**{**case.__dict__, "body": np.ascontiguousarray(body2)})
    ref = oracle_lib.forcing(case2, mask=m_np)
    for k in ("u", "f_tot", "S", "T"):
        assert rel_err(got[k], ref[k]) <= 1e-12, k


def test_graph_profiled_as_one_class():
    dev = require_gpu()
    case = synth.small_case(73, n=(36, 36, 40), periodic=(1, 1, 0), n_iter=2)
    _, mk = _mask(case, dev)
    plan, D = _setup(case, "f32")
    u0 = D["u"].clone()
    _run(plan, D, u0, mk, True)
    plan.profile(True)
    for _ in range(3):
        _run(plan, D, u0, mk, True)
    st = plan.stats()
    plan.profile(False)
    assert st["kernel_launches"]["graph"] == 3
    assert st["kernel_ms"]["graph"] > 0.0
    assert st["kernel_launches"]["interp"] == 0


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tune_keeps_inputs_and_results(oracle_lib, precision):
    import torch
    dev = require_gpu()
    case = synth.make_case("suspension_128")
    m_np, mk = _mask(case, dev)
    plan, D = _setup(case, precision)
    u_before = D["u"].clone()
    D["f"].fill_(0.25)
    f_before = D["f"].clone()
    st = plan.tune(D["u"], D["f"], D["xp"], D["up"], D["wp"], mask=mk)
    plan.check("tune")
    print(f"{precision}: tuned tile {st['tile']} block {st['block']} persistent "
          f"{st['persistent']}", flush=True)
    assert torch.equal(D["u"], u_before) and torch.equal(D["f"], f_before)
    assert all(4 <= t <= 32 for t in st["tile"])
    assert st["block"] in (64, 128, 256) and st["persistent"] in (0, 1)
    got = _run(plan, D, u_before, mk, False)
    got_g = _run(plan, D, u_before, mk, True)
    ref = oracle_lib.forcing(case, mask=m_np)
    tol = dict(f64=dict(u=1e-12, f_tot=1e-12, S=1e-12, T=1e-12),
               f32=dict(u=1e-4, f_tot=1e-4, S=1e-4, T=1e-4))[precision]
    for res in (got, got_g):
        for k in ("u", "f_tot", "S", "T"):
            e = rel_err(res[k], ref[k])
            assert e <= tol[k], f"{k}: {e:.3e}"


@pytest.mark.parametrize("n", [(41, 37, 45), (48, 40, 44)])
@pytest.mark.parametrize("tile", [(8, 8, 8), (32, 16, 4), (16, 8, 16), (4, 4, 4), (12, 16, 8)])
def test_tile_shapes_parity(oracle_lib, tile, n):
    """Tile shapes on a grid whose x extent is not a multiple of 4 (element
    staging and write-out) and on one that is (16-byte packets)."""
    dev = require_gpu()
    case = synth.small_case(74, n=n, periodic=(1, 1, 0), n_iter=2, touch=0.4)
    m_np, mk = _mask(case, dev)
    ref = oracle_lib.forcing(case, mask=m_np)
    for precision, tol in (("f64", 1e-12), ("f32", 1e-4)):
        plan, D = _setup(case, precision)
        plan.set_tiles(*tile)
        got = _run(plan, D, D["u"].clone(), mk, False)
        print(precision, tile, plan.stats()["tile"], flush=True)
        for k in ("u", "f_tot", "S", "T"):
            e = rel_err(got[k], ref[k])
            assert e <= tol, f"{precision} tile {tile} {k}: {e:.3e}"


@pytest.mark.parametrize("tile", [(4, 4, 4), (60, 4, 8), (32, 8, 8)])
def test_tile_shapes_parity_four_point(oracle_lib, tile):
    """The four-point delta (a 4-node support on 4-node tile edges, and the
    whole x extent in one tile) with walls in z; the grid's edges are
    multiples of 4, so the requested shapes are used as they are."""
    dev = require_gpu()
    case = synth.small_case(76, n=(48, 40, 44), periodic=(1, 1, 0), n_iter=2, touch=0.4)
    case.params.update(kernel=4, eps_sep=2.0, lub_C=4.0, gap_cut=4.0)
    m_np, mk = _mask(case, dev)
    ref = oracle_lib.forcing(case, mask=m_np, kernel=4)
    for precision, tol in (("f64", 1e-12), ("f32", 1e-4)):
        plan, D = _setup(case, precision)
        plan.set_tiles(*tile)
        got = _run(plan, D, D["u"].clone(), mk, False)
        print(precision, tile, plan.stats()["tile"], flush=True)
        assert plan.stats()["tile"] == (min(tile[0], 48),) + tuple(tile[1:])
        for k in ("u", "f_tot", "S", "T"):
            e = rel_err(got[k], ref[k])
            assert e <= tol, f"{precision} tile {tile} {k}: {e:.3e}"


def test_set_tiles_rejects_bad_shapes():
    from paper_2109_03972_amd import ibmx
    require_gpu()
    case = synth.small_case(75, n=(36, 36, 40), periodic=(1, 1, 0), n_iter=1)
    plan, _ = _setup(case, "f64")
    before = plan.stats()["tile"]
    for bad in ((3, 16, 16), (16, 16, 65), (61, 8, 8)):
        with pytest.raises(ibmx.IbmxError):
            plan.set_tiles(*bad)
        assert plan.stats()["tile"] == before


@pytest.mark.parametrize("kernel,tile", [(3, (8, 8, 8)), (4, (32, 8, 8))])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_launch_forms_bit_identical(oracle_lib, precision, kernel, tile):
    """Every workgroup size the tuner tries (64, 128, 256 threads: the markers
    a tile's workgroup takes at once) and both launch forms (one workgroup
    per tile; a persistent grid looping over the tiles) give the same bits,
    eager and replayed as a graph, and match the oracle; with both delta
    kernels."""
    import torch
    dev = require_gpu()
    case = synth.small_case(76, n=(44, 40, 46), periodic=(1, 1, 0), n_iter=3, touch=0.4)
    if kernel == 4:
        case.params.update(kernel=4, eps_sep=2.0, lub_C=4.0, gap_cut=4.0)
    m_np, mk = _mask(case, dev)
    ref = oracle_lib.forcing(case, mask=m_np)
    plan, D = _setup(case, precision)
    plan.set_tiles(*tile)
    u0 = D["u"].clone()
    resid = torch.zeros(int(case.params["n_iter"]) + 1, dtype=torch.float64, device=dev)
    base = _run(plan, D, u0, mk, False, resid)
    tol = 1e-12 if precision == "f64" else 1e-4
    for k in ("u", "f_tot", "S", "T", "resid"):
        assert rel_err(base[k], ref[k]) <= tol, k
    for block in (64, 128, 256):
        for persistent in (False, True):
            plan.set_launch(block, persistent)
            st = plan.stats()
            assert (st["block"], st["persistent"]) == (block, int(persistent))
            for graph in (False, True):
                got = _run(plan, D, u0, mk, graph, resid)
                for k in ("u", "f_tot", "S", "T", "resid"):
                    np.testing.assert_array_equal(
                        got[k], base[k], err_msg=f"block {block} persistent {persistent} {k}")
    from paper_2109_03972_amd import ibmx
    for bad in ((32, 0), (512, 0), (256, 2)):
        with pytest.raises(ibmx.IbmxError):
            plan.set_launch(*bad)
