"""The library's own kernel and runtime sources, compiled for the host under
AddressSanitizer + UndefinedBehaviorSanitizer (tests/cpu_emu), run small
cases of every code path and are compared with the FP64 oracle.  Any read
or write outside the caller's workspace or tensors, any undefined integer
or float-to-int conversion, and any divergent barrier aborts the run.

This is the CPU check of every kernel's indexing and launch shape before it
runs on a GPU; it is not a fallback (the package never loads it)."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as wl
from emu import run_case, run_cases
from helpers import compare_fields, oracle_dev, weights

# The longest cases (tens of seconds each under the sanitizers) start as
# background processes when the module's first test runs; their tests
# collect the results.


def _rest_case():
    ps = [wl.Params(dim=2, nx=40, ny=24, tau=1.0, sigma=0.004, theta_eq_deg=90.0, xi=2.0),
          wl.Params(dim=2, nx=48, ny=20, tau=0.8, sigma=0.02, theta_eq_deg=60.0, xi=2.0),
          wl.Params(dim=2, nx=32, ny=8, tau=0.9, wetting=False)]
    qs = [wl.cap_polygon(6.0, 90.0, 2.0, 40, 20.0), wl.cap_polygon(6.0, 90.0, 2.0, 40, 24.0), None]
    return ps, qs


def _tiny3d_case():
    p = wl.Params(dim=3, nx=20, ny=18, nz=12, bc=(0, 0, 1), tau=0.8, sigma=0.005,
                  theta_eq_deg=70.0, xi=2.0)
    V, T = wl.cap_mesh(5.0, 90.0, 2.0, 3, (10.0, 9.0))
    return p, V, T


def _coarse3d_case():
    p = wl.Params(dim=3, nx=24, ny=22, nz=14, bc=(0, 0, 1), tau=0.9, sigma=0.006,
                  theta_eq_deg=100.0, xi=2.0)
    V, T = wl.cap_mesh(9.0, 90.0, 2.0, 4, (1.0, 11.0))
    return p, V, T


def _visc3d_case():
    """Coarse cap across the periodic x edge, viscosity ratio 4."""
    p = wl.Params(dim=3, nx=24, ny=22, nz=14, bc=(0, 0, 1), tau=0.7, sigma=0.006,
                  theta_eq_deg=80.0, xi=2.0, lam=4.0)
    V, T = wl.cap_mesh(7.0, 90.0, 2.0, 4, (1.5, 10.3))
    return p, V, T


def _contact2d_case():
    p = wl.Params(dim=2, nx=80, ny=40, tau=0.8, sigma=0.006, theta_eq_deg=50.0, xi=2.0)
    q = wl.cap_polygon(12.0, 90.0, 2.0, 80, 40.0)
    return p, q, (o.h_star(p.xi), 0.05 * 12.0)


def _elastic3d_case():
    p = wl.Params(dim=3, nx=20, ny=18, nz=12, bc=(0, 0, 1), tau=0.8, sigma=0.005,
                  theta_eq_deg=60.0, xi=2.0, shear=0.02)
    V, T = wl.cap_mesh(5.0, 90.0, 2.0, 3, (10.0, 9.0))
    return p, V, T


def _blowup_case():
    p = wl.Params(dim=2, nx=64, ny=32, tau=1.0, sigma=50.0, theta_eq_deg=60.0, xi=2.0)
    q = wl.cap_polygon(8.0, 90.0, 2.0, 40, 32.0)
    return p, q


def _background_jobs():
    ps, qs = _rest_case()
    p3, V3, T3 = _tiny3d_case()
    pc, Vc, Tc = _coarse3d_case()
    pb, qb = _blowup_case()
    pv, Vv, Tv = _visc3d_case()
    p2, q2, c2 = _contact2d_case()
    pe, Ve, Te = _elastic3d_case()
    return {
        "contact2d": dict(params_list=[p2], nodes_list=[q2], steps=(3,), contact=c2),
        "contact3d": dict(params_list=[p3], nodes_list=[V3], tris_list=[T3], steps=(2,),
                          contact=(2.7, 0.02 * 5.0)),
        "elastic3d": dict(params_list=[pe], nodes_list=[Ve], tris_list=[Te], steps=(1, 3), graph_steps=2),
        "visc3d": dict(params_list=[pv], nodes_list=[Vv], tris_list=[Tv], steps=(1, 2), graph_steps=2,
                       masks=True),
        "rest": dict(params_list=ps, nodes_list=qs, steps=(0,), rest=(2e-3, 4, 2, 60), graph_steps=2),
        "tiny3d": dict(params_list=[p3], nodes_list=[V3], tris_list=[T3], steps=(3,), graph_steps=2),
        # blocks in the storage order of their tiles, flat form
        "tiny3d_storage_order": dict(params_list=[p3], nodes_list=[V3], tris_list=[T3], steps=(3,),
                                     graph_steps=2, shape=31),
        "coarse3d": dict(params_list=[pc], nodes_list=[Vc], tris_list=[Tc], steps=(2,), graph_steps=2),
        "coarse3d_direct": dict(params_list=[pc], nodes_list=[Vc], tris_list=[Tc], steps=(2,),
                                graph_steps=2, direct_chunks=True),
        "blowup": dict(params_list=[pb], nodes_list=[qb], steps=(50,)),
    }


@pytest.fixture(scope="module", autouse=True)
def background():
    from concurrent.futures import ThreadPoolExecutor
    jobs = _background_jobs()
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        yield {k: ex.submit(run_case, **kw) for k, kw in jobs.items()}


def test_droplet_2d_graph_and_tiles():
    """Three tile shapes and a non-temporal-load variant; graph replays of 2
    steps plus direct launches, the timed schedule, and no graphs."""
    W = wl.droplet_2d_small()
    cases = ((0, 2), (4, 2), (2, 0), (10, 2), (13, 2))
    outs = run_cases([dict(params_list=[W.params], nodes_list=[W.nodes], steps=(5, 4), shape=shape,
                           graph_steps=gs, timing=(shape == 4)) for shape, gs in cases])
    r = o.run(W.params, W.nodes, 9)
    for (shape, gs), out in zip(cases, outs):
        g = out[0]
        drho, du, dq = compare_fields(g, r, 2, f"emu tile{shape}")
        assert g["status"] == 0
        assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7
        assert abs(g["diag"]["mass"] - r["f"].sum()) < 1e-6


@pytest.mark.parametrize("shape", [5, 14])
def test_ragged_box_and_periodic_crossing(shape):
    """A box whose rows are not a multiple of 64 cells, with a tiled and a
    flat lattice-kernel variant (in the flat one a wavefront spans rows)."""
    p = wl.Params(dim=2, nx=101, ny=37, tau=0.8, sigma=0.008, theta_eq_deg=110.0, xi=2.0)
    q = wl.cap_polygon(10.0, 95.0, 2.0, 70, 2.0)
    g = run_case([p], [q], steps=(7,), shape=shape, graph_steps=2)[0]
    r = o.run(p, q, 7)
    drho, du, dq = compare_fields(g, r, 2, "emu ragged")
    assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7


def test_batch_with_fluid_only_member():
    ps = [wl.Params(dim=2, nx=96, ny=40, tau=0.7, sigma=0.006, theta_eq_deg=40.0, xi=2.0),
          wl.Params(dim=2, nx=70, ny=33, tau=1.3, sigma=0.009, theta_eq_deg=140.0, xi=2.0),
          wl.Params(dim=2, nx=64, ny=8, tau=0.9, wetting=False)]
    qs = [wl.cap_polygon(12.0, 90.0, 2.0, 94, 48.0), wl.cap_polygon(9.0, 90.0, 2.0, 71, 35.0),
          None]
    # plain, then timed direct launches with a frozen member that must not move
    out, out_t = run_cases([dict(params_list=ps, nodes_list=qs, steps=(6,), graph_steps=2),
                            dict(params_list=ps, nodes_list=qs, steps=(3, 3), timing=True,
                                 inactive=(1,))])
    for d in range(2):
        r = o.run(ps[d], qs[d], 6)
        drho, du, dq = compare_fields(out[d], r, 2, f"emu batch{d}")
        assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7
    assert np.all(out[2]["fdev"] == 0)
    out = out_t
    r = o.run(ps[0], qs[0], 6)
    drho, du, dq = compare_fields(out[0], r, 2, "emu batch timed")
    assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7
    assert np.array_equal(out[1]["q"], qs[1]) and np.all(out[1]["fdev"] == 0)


def test_node_respacing_2d_single_and_batch():
    """Tangential re-spacing of unevenly spaced outlines (every third node
    removed along part of the arc), for a lone droplet and inside a batch
    (the two ring lookups of the fused node kernel), through the first-step,
    fused and last-step node kernels; the oracle's run with the same rate
    must agree, and the re-spacing must move the nodes."""
    import dataclasses
    p1 = wl.Params(dim=2, nx=96, ny=40, tau=0.7, sigma=0.006, theta_eq_deg=40.0, xi=2.0, respace=0.4)
    p2 = wl.Params(dim=2, nx=70, ny=33, tau=1.3, sigma=0.009, theta_eq_deg=140.0, xi=2.0, respace=0.25)
    q1 = np.delete(wl.cap_polygon(12.0, 90.0, 2.0, 94, 48.0), list(range(10, 40, 3)), axis=0)
    q2 = np.delete(wl.cap_polygon(9.0, 90.0, 2.0, 71, 35.0), list(range(5, 30, 3)), axis=0)
    lone, batch = run_cases([dict(params_list=[p1], nodes_list=[q1], steps=(5, 4), graph_steps=2),
                             dict(params_list=[p1, p2], nodes_list=[q1, q2], steps=(5, 4), graph_steps=2)])
    r1 = o.run(p1, q1, 9)
    r0 = o.run(dataclasses.replace(p1, respace=0.0), q1, 9)
    assert np.max(np.abs(r1["q"] - r0["q"])) > 1e-2
    for g, r, name in ((lone[0], r1, "lone"), (batch[0], r1, "batch0"), (batch[1], o.run(p2, q2, 9), "batch1")):
        drho, du, dq = compare_fields(g, r, 2, f"emu respace {name}")
        assert g["status"] == 0
        assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7


def test_two_viscosities_2d_across_periodic_edge():
    """Viscosity ratio 10, ragged box, droplet across the periodic x edge:
    the classification at the initial and the final node positions equals
    the oracle's, and 7 steps (graph replays and direct launches) match the
    oracle's run."""
    p = wl.Params(dim=2, nx=101, ny=37, tau=0.7, sigma=0.008, theta_eq_deg=110.0, xi=2.0, lam=10.0)
    q = wl.cap_polygon(10.0, 95.0, 2.0, 70, 2.0)
    g = run_case([p], [q], steps=(3, 4), graph_steps=2, masks=True)[0]
    assert g["status"] == 0, g["message"]
    ref = o.reference_point(q)
    m0 = o.inside_mask(p, q, ref=ref)
    assert np.array_equal(g["inside0"], m0) and m0.sum() > 150
    assert np.array_equal(g["inside1"], o.inside_mask(p, g["q"], ref=ref))
    r = o.run(p, q, 7)
    drho, du, dq = compare_fields(g, r, 2, "emu two viscosities 2d")
    assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7
    # the ratio matters at this tolerance
    p1 = wl.Params(**{**p.to_dict(), "lam": 1.0})
    r1 = o.run(p1, q, 7)
    assert np.max(np.abs(r1["U"] - r["U"])) > 1e-4


def test_two_viscosities_batch_mixed():
    """A batch with a one-fluid droplet, a droplet with ratio 0.2 and a
    frozen droplet with ratio 5, stepped an odd number of steps per call."""
    ps = [wl.Params(dim=2, nx=60, ny=30, tau=0.8, sigma=0.006, theta_eq_deg=50.0, xi=2.0),
          wl.Params(dim=2, nx=50, ny=28, tau=1.1, sigma=0.009, theta_eq_deg=120.0, xi=2.0, lam=0.2),
          wl.Params(dim=2, nx=40, ny=24, tau=0.9, sigma=0.007, theta_eq_deg=90.0, xi=2.0, lam=5.0)]
    qs = [wl.cap_polygon(8.0, 90.0, 2.0, 50, 30.0), wl.cap_polygon(7.0, 90.0, 2.0, 44, 25.0),
          wl.cap_polygon(6.0, 90.0, 2.0, 40, 20.0)]
    out = run_case(ps, qs, steps=(3, 2), graph_steps=2, inactive=(2,), masks=True)
    for d in range(2):
        r = o.run(ps[d], qs[d], 5)
        drho, du, dq = compare_fields(out[d], r, 2, f"emu mixed{d}")
        assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7
        assert np.array_equal(out[d]["inside0"], o.inside_mask(ps[d], qs[d]))
    assert np.array_equal(out[2]["q"], qs[2]) and np.all(out[2]["fdev"] == 0)
    assert np.array_equal(out[2]["inside1"], o.inside_mask(ps[2], qs[2]))


def test_too_many_crossings_on_a_row_is_reported():
    """A comb-shaped outline crosses some rows 24 times: the step reports
    IBLB_ELIMIT and drops the extra crossings (no access beyond the
    tables)."""
    pts = [(2.0, 2.0), (56.0, 2.0), (56.0, 4.0)]
    for k in range(11, -1, -1):
        pts += [(6.0 + 4 * k, 4.0), (6.0 + 4 * k, 20.0), (4.0 + 4 * k, 20.0), (4.0 + 4 * k, 4.0)]
    q = np.array(pts + [(2.0, 4.0)]) + np.array([0.25, 0.125])
    p = wl.Params(dim=2, nx=64, ny=32, tau=0.8, sigma=0.005, wetting=False, lam=3.0)
    g = run_case([p], [q], steps=(2,), graph_steps=0)[0]
    assert g["status"] == -5 and "crossings" in g["message"]


def test_contact_radius_protocols(background):
    """Both protocols on the device's final positions against the oracle's
    formulas on the same positions (2D, and the tiny 3D cap)."""
    p, q, (zc, tol) = _contact2d_case()
    g = background["contact2d"].result()[0]
    ri, rii, n = g["contact"]
    assert n == 2
    assert abs(ri - o.contact_radius_2d(g["q"], zc)) < 1e-12 * ri
    assert abs(rii - o.contact_radius_flat_2d(g["q"], tol)) < 1e-12 * rii
    p3, V, T = _tiny3d_case()
    g3 = background["contact3d"].result()[0]
    ri, rii, n = g3["contact"]
    assert n > 10
    assert abs(ri - o.contact_radius_3d(g3["q"], T, 2.7)) < 1e-12 * ri
    assert abs(rii - o.contact_radius_flat_3d(g3["q"], T, 0.02 * 5.0)) < 1e-12 * rii


def test_elastic_interface_3d(background):
    """Coarse cap with an elastic interface (shear modulus 0.02, reference
    = the initial mesh): 4 steps (graph replays and direct launches) against
    the oracle."""
    p, V, T = _elastic3d_case()
    g = background["elastic3d"].result()[0]
    assert g["status"] == 0, g["message"]
    r = o.run(p, V, 4, tris=T)
    drho, du, dq = compare_fields(g, r, 3, "emu elastic 3d")
    assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7
    assert np.max(np.abs(g["phi"] - r["phi"])) <= 1e-6 * np.max(np.abs(r["phi"]))
    # the shear term matters at this tolerance
    p0 = wl.Params(**{**p.to_dict(), "shear": 0.0})
    r0 = o.run(p0, V, 4, tris=T)
    assert np.max(np.abs(r0["phi"] - r["phi"])) > 1e-3 * np.max(np.abs(r["phi"]))


def test_droplet_wider_than_the_window_is_reported():
    p = wl.Params(dim=2, nx=40, ny=32, tau=0.8, sigma=0.004, wetting=False, lam=2.0)
    t = 2.0 * np.pi * np.arange(120) / 120
    q = np.stack([20.0 + 22.0 * np.cos(t), 16.0 + 6.0 * np.sin(t)], axis=1)
    g = run_case([p], [q], steps=(1,), graph_steps=0)[0]
    assert g["status"] == -5 and "window" in g["message"]


def test_two_viscosities_3d(background):
    p, V, T = _visc3d_case()
    g = background["visc3d"].result()[0]
    assert g["status"] == 0, g["message"]
    ref = o.reference_point(V)
    m0 = o.inside_mask(p, V, T, ref=ref)
    assert np.array_equal(g["inside0"], m0) and m0.sum() > 300
    assert np.array_equal(g["inside1"], o.inside_mask(p, g["q"], T, ref=ref))
    r = o.run(p, V, 3, tris=T)
    drho, du, dq = compare_fields(g, r, 3, "emu two viscosities 3d")
    assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7


def test_droplet_3d_tiny(background):
    p, V, T = _tiny3d_case()
    r = o.run(p, V, 3, tris=T)
    for key in ("tiny3d", "tiny3d_storage_order"):
        g = background[key].result()[0]
        drho, du, dq = compare_fields(g, r, 3, f"emu 3d {key}")
        assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7
        assert abs(g["diag"]["volume"] - o.volume_3d(r["q"], T)) < 1e-9 * abs(g["diag"]["volume"])


def test_droplet_3d_coarse_mesh_across_periodic_edge(background):
    """Coarse cap centred on the periodic x edge, spreading boxes that wrap
    around the periodic axis.  The second build has the host cut plain runs
    of the chunk size (16 vertices) without the box budget, so some chunks
    overflow the LDS box and add straight to global memory next to chunks
    that fit."""
    p, V, T = _coarse3d_case()
    r = o.run(p, V, 2, tris=T)
    assert np.min(r["q"][:, 0]) < 0.0
    for key in ("coarse3d", "coarse3d_direct"):
        out = background[key].result()
        drho, du, dq = compare_fields(out[0], r, 3, f"emu 3d periodic {key}")
        assert drho <= 1e-6 and du <= 1e-5 and dq <= 1e-7


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_streaming_bit_exact_all_storages(storage):
    for dim, (nx, ny, nz), bc in ((2, (37, 9, 1), (0, 1, 0)), (3, (9, 5, 4), (1, 0, 1))):
        Q = 9 if dim == 2 else 19
        w = weights(dim)
        dev = wl.tagged_deviation(Q, nx * ny * nz, 5).reshape(Q, nz, ny, nx)
        p = wl.Params(dim=dim, nx=nx, ny=ny, nz=nz, bc=bc, tau=math.inf, wetting=False)
        f = w[:, None, None, None] + dev
        for _ in range(3):
            f, _, _ = o.lb_step(dim, nx, ny, nz, bc, math.inf, f, None)
        k = np.rint((f - w[:, None, None, None]) * 1024.0)
        # default variant (tiles in runs per XCD) and a tiled one in storage order
        for shape in (None, 17):
            g = run_case([p], steps=(3,), storage=storage, f0dev=[dev], graph_steps=2, shape=shape)[0]
            assert np.array_equal(g["fdev"], k / 1024.0), (dim, shape)


def test_prescribed_force_field():
    nx, ny, nz = 23, 7, 1
    w = weights(2)
    rng = np.random.default_rng(9)
    dev = 1e-2 * w[:, None, None, None] * rng.standard_normal((9, nz, ny, nx))
    F = np.zeros((3, nz, ny, nx))
    F[:2] = 1e-4 * rng.standard_normal((2, nz, ny, nx))
    p = wl.Params(dim=2, nx=nx, ny=ny, bc=(0, 1, 0), tau=0.7, wetting=False)
    g = run_case([p], steps=(4,), f0dev=[dev], forces=[F])[0]
    r = o.run(p, None, 4, f0=w[:, None, None, None] + dev, F_fixed=F)
    assert np.max(np.abs(g["fdev"] - oracle_dev(2, r["f"]))) <= 1e-8
    assert np.max(np.abs(g["U"] - r["U"][:2])) <= 1e-8


def test_blow_up_is_reported_without_undefined_behaviour(background):
    """Huge surface tension: speeds and then positions become non-finite.
    The step reports IBLB_EUNSTABLE and no tap index is formed from a
    non-finite coordinate."""
    g = background["blowup"].result()[0]
    assert g["status"] == -4
    assert g["diag"]["status"] == -4


def test_run_to_rest_freezes_settled_droplets(background):
    """A loose tolerance so that the tiny cases settle within a few checks:
    each droplet's frozen state equals the oracle after its reported step
    count; the fluid-only member is ignored."""
    ps, qs = _rest_case()
    out = background["rest"].result()
    assert out[2]["rest_steps"] == 0
    for d in range(2):
        n = out[d]["rest_steps"]
        assert n > 0 or n == -1
        r = o.run(ps[d], qs[d], n if n > 0 else 60)
        assert np.max(np.abs(out[d]["q"] - r["q"])) <= 1e-7
    assert out[0]["rest_steps"] > 0


def _bf16(a):
    """Round to bf16 (nearest even) and back, like the network's operands."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("widths,batch", [([4, 40, 33, 70], 37), ([4, 40, 70], 300), ([4, 64, 40, 520], 300)])
def test_network_kernels_against_reference(widths, batch):
    """Ragged sizes (K = 4, widths not multiples of the 32x32 tiles, batch
    not a multiple of 64) through forward, gradients and one Adam step; the
    batch of 300 splits the weight-gradient products over K.  Widths that
    are multiples of 8 take the 16-byte operand fetches; 520 outputs give
    the input-side product of the last layer five K panels of 128, the last
    one partial."""
    from emu import run_mlp
    from oracle import mlp
    rng = np.random.default_rng(3)
    p = mlp.init_params(widths, 7)
    x = rng.standard_normal((batch, 4))
    t = 0.3 * rng.standard_normal((batch, widths[-1]))
    y, g, loss, pa = run_mlp(widths, p, x, t, lr=1e-3)
    yo, _ = mlp.forward(p, widths, x)
    lo, go = mlp.loss_and_grad(p, widths, x, t)
    assert np.max(np.abs(y - yo)) <= 3e-2 * np.max(np.abs(yo))
    assert abs(loss - lo) <= 2e-2 * lo
    cos = float(np.dot(g, go) / (np.linalg.norm(g) * np.linalg.norm(go)))
    assert cos >= 0.999 and np.linalg.norm(g - go) <= 2e-2 * np.linalg.norm(go)
    # one Adam step from the library's own gradient
    ref = mlp.Adam(len(p)).step(p.astype(np.float32).astype(np.float64), g.astype(np.float64), 1e-3)
    assert np.max(np.abs(pa - ref)) <= 1e-6
