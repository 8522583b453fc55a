"""CPU checks of the C ABI library: it loads, exports every function declared
in include/mcs.h, and its host planning (topology, dof counts, colouring,
multigrid plan, error codes) agrees with the oracle and the definitions.
No compute calls (no GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2207_08481_amd", "libmcs.so")
HEADER = os.path.join(ROOT, "include", "mcs.h")

needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libmcs.so not built")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mcs_[a-z_0-9]+)\s*\(", txt)))


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    from paper_2207_08481_amd.mcs import SYMBOLS
    assert sorted(SYMBOLS) == names


@needs_lib
@pytest.mark.parametrize("d,n,k", [(2, 4, 2), (2, 3, 4), (3, 2, 2), (3, 3, 3), (3, 2, 5), (3, 3, 1)])
def test_plan_sizes_and_topology(d, n, k):
    from paper_2207_08481_amd import Problem
    from oracle.topology import Topology
    from oracle.element import expected_dims
    mesh = W.unit_square_mesh(n) if d == 2 else W.unit_cube_mesh(n)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, k)
    topo = Topology(mesh.vertices, mesh.elements)
    dims = expected_dims(d, k)
    i = pb.info
    assert i.n_bub == dims["n_bub"] and i.n_F == dims["n_F"] and i.n_hat == dims["n_hat"]
    assert i.n_p == dims["n_p"]
    assert i.n_free_facets == topo.n_free_facets
    ne = mesh.n_elements
    assert i.n_dof == ne * dims["n_bub"] + topo.n_free_facets * dims["n_fb"] + ne * dims["n_p"]
    assert i.n_p1_dofs == d * len(topo.free_vertices)
    colour, eff = pb.topology()
    assert np.array_equal(colour, topo.colour)
    ff = np.where(topo.free_facet_of[topo.elem_facets] >= 0, topo.free_facet_of[topo.elem_facets], -1)
    assert np.array_equal(eff, ff)
    # colouring validity: facets of one element have distinct colours
    for e in range(ne):
        cs = [colour[g] for g in eff[e] if g >= 0]
        assert len(cs) == len(set(cs))
    assert i.workspace_bytes > 0


@needs_lib
def test_paper_scale_dof_count():
    """32^3 x 6 tets, k = 4: 26,327,040 free dofs (2 n_fb + n_bub + n_p per tet asymptotically)."""
    from paper_2207_08481_amd import Problem
    mesh = W.unit_cube_mesh(32)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 4)
    assert pb.info.n_dof == 26327040
    assert pb.info.n_colours == 4
    assert pb.info.n_mg_levels == 4


@needs_lib
def test_multigrid_levels_rule():
    from paper_2207_08481_amd import Problem
    mesh = W.unit_cube_mesh(16)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 2)
    assert pb.info.n_mg_levels == 3        # 15^3*3 = 10125 -> 7^3*3 = 1029 > 512 -> 3^3*3 = 81
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, coarse_max=2000)
    assert pb.info.n_mg_levels == 2


@needs_lib
def test_error_codes():
    from paper_2207_08481_amd.mcs import Problem, MCSError
    mesh = W.unit_cube_mesh(2)
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, mesh.elements, mesh.lattice, 0)
    assert ex.value.status == -1
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, mesh.elements, mesh.lattice, 6)
    assert ex.value.status == -10
    bad = mesh.elements.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, bad, mesh.lattice, 2)
    assert ex.value.status == -2
    flat = mesh.vertices.copy()
    flat[:, 2] = 0.0
    with pytest.raises(MCSError) as ex:
        Problem(flat, mesh.elements, mesh.lattice, 2)
    assert ex.value.status == -2
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, mesh.elements, (3, 3, 4), 2)
    assert ex.value.status == -2
    nanv = mesh.vertices.copy()
    nanv[3, 0] = np.nan
    with pytest.raises(MCSError) as ex:
        Problem(nanv, mesh.elements, mesh.lattice, 2)
    assert ex.value.status == -1
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, precision=3)
    assert ex.value.status == -1
    # smoother options: 0..3; the full-system variant needs precision 0 and
    # blocks of at most 64 dofs (3D: k <= 3)
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, smoother=4)
    assert ex.value.status == -1
    Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, smoother=3, precision=1).close()
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, precision=1, smoother=2)
    assert ex.value.status == -10
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, mesh.elements, mesh.lattice, 4, smoother=2)
    assert ex.value.status == -10
    Problem(mesh.vertices, mesh.elements, mesh.lattice, 3, smoother=2).close()


def test_full_system_blocks_and_colouring():
    """The planner's blocks of the full-system variant: one per facet of the
    mesh (Dirichlet facets included), coloured greedily in canonical facet
    order exactly as the oracle colours them."""
    from paper_2207_08481_amd.mcs import Problem
    from oracle.topology import Topology
    for mesh in (W.unit_square_mesh(3), W.unit_cube_mesh(2)):
        pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, smoother=2)
        topo = Topology(mesh.vertices, mesh.elements)
        # greedy colouring of all facets (oracle rule, restated here on the topology)
        colour = -np.ones(topo.n_facets, dtype=int)
        for f in range(topo.n_facets):
            used = {colour[f2] for (t, _i) in topo.facet_neighbors[f] for f2 in topo.elem_facets[t]
                    if f2 != f and colour[f2] >= 0}
            c = 0
            while c in used:
                c += 1
            colour[f] = c
        assert np.array_equal(pb.full_colouring(), colour)
        pb.close()


@needs_lib
def test_unbound_calls_are_refused():
    from paper_2207_08481_amd.mcs import Problem, load_library
    import ctypes as C
    mesh = W.unit_square_mesh(2)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 2)
    lib = load_library()
    rc = lib.mcs_condense(pb._h, C.c_void_p(0))
    assert rc == -8          # not bound to a workspace
    rc = lib.mcs_bind(pb._h, C.c_void_p(0), 0, C.c_void_p(0))
    assert rc == -3          # workspace missing


@needs_lib
def test_batch_plan_groups_members_and_sizes():
    """mcs_batch_plan groups members by (dimension, order), gives each member
    the sizes of its own plan, and sums them."""
    from paper_2207_08481_amd import Batch, Problem
    specs = [(3, 2, 2), (2, 3, 3), (3, 3, 2), (3, 2, 4), (2, 2, 3)]
    meshes, orders, singles = [], [], []
    for d, n, k in specs:
        m = W.unit_square_mesh(n) if d == 2 else W.unit_cube_mesh(n)
        meshes.append((m.vertices, m.elements, m.lattice))
        orders.append(k)
        singles.append(Problem(m.vertices, m.elements, m.lattice, k))
    b = Batch(meshes, orders)
    assert b.info.n_problems == len(specs)
    assert b.info.n_groups == 3                 # (3,2), (2,3), (3,4)
    assert b.info.n_dof_total == sum(p.n_dof for p in singles)
    assert b.info.workspace_bytes > sum(0 for _ in singles)
    for mi, p in zip(b.members, singles):
        for f in ("n_dof", "n_bubble_dofs", "n_facet_dofs", "n_pressure_dofs", "n_p1_dofs", "n_free_facets",
                  "n_colours", "n_mg_levels"):
            assert getattr(mi, f) == getattr(p.info, f), f


@needs_lib
def test_batch_plan_errors_name_the_member():
    from paper_2207_08481_amd.mcs import Batch, MCSError
    m = W.unit_cube_mesh(2)
    with pytest.raises(MCSError) as ex:
        Batch([(m.vertices, m.elements, m.lattice)] * 3, [2, 3, 7])
    assert ex.value.status == -10 and "member 2" in str(ex.value)
    with pytest.raises(MCSError) as ex:
        Batch([(m.vertices, m.elements, (3, 3, 4))], [2])
    assert ex.value.status == -2


@needs_lib
def test_batch_members_recipe():
    """Batch member recipe: sizes within the log-uniform range, orders from
    the given set, seeded."""
    ms = W.batch_members(256, seed=5)
    assert len(ms) == 256
    ns = np.array([m["n"] for m in ms])
    assert ns.min() >= 4 and ns.max() <= 16
    assert set(m["k"] for m in ms) == {2, 3, 4}
    assert ms == W.batch_members(256, seed=5)


def test_outlet_plan_matches_oracle_topology():
    """Outlet faces (face_bc = 1): the planner's free facets (interior and
    outlet, canonical order), their colours, the element -> free facet map and
    the free P1 vertices equal the oracle's topology."""
    from paper_2207_08481_amd.mcs import Problem
    from oracle.topology import Topology
    for cells, fb in (((4, 3), [0, 1, 0, 0]), ((2, 2, 2), [0, 1, 0, 0, 0, 0]), ((3, 2, 2), [1, 0, 0, 0, 0, 1])):
        mesh = W.box_mesh(cells, (1.0,) * len(cells))
        d = len(cells)
        pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, face_bc=fb)
        topo = Topology(mesh.vertices, mesh.elements, fb)
        assert pb.info.n_free_facets == topo.n_free_facets
        assert pb.info.n_p1_dofs == d * len(topo.free_vertices)
        colour, elem_ff = pb.topology()
        assert np.array_equal(colour, topo.colour)
        ref = topo.free_facet_of[topo.elem_facets]
        assert np.array_equal(elem_ff.reshape(ref.shape), ref)
        pb.close()


def test_outlet_errors():
    from paper_2207_08481_amd.mcs import Problem, MCSError, Batch
    mesh = W.box_mesh((2, 2), (1.0, 1.0))
    with pytest.raises(MCSError) as ex:
        Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, face_bc=[0, 2, 0, 0])
    assert ex.value.status == -1
    with pytest.raises(MCSError) as ex:
        Batch([(mesh.vertices, mesh.elements, mesh.lattice)], [2], face_bcs=[[0, 1, 0, 0]])
    assert ex.value.status == -10


def test_launch_config_setter_validates():
    """mcs_set_launch_config takes 1 or 2 facet blocks per workgroup and a
    grid cap >= 0 for FP64 or FP32 work precision; anything else is refused
    with MCS_ERR_ARG and leaves the shape unchanged (host only)."""
    from paper_2207_08481_amd.mcs import F32, F64, MCSError, Problem
    mesh = W.unit_cube_mesh(1)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 3)
    pb.set_launch_config(2, 64, F32)
    assert pb.launch_config(F32) == {"facets_per_block": 2, "grid_cap": 64, "us_per_launch": 0.0}
    for fpb, cap, dt in ((3, 0, F64), (0, 0, F64), (1, -1, F64), (1, 0, 7)):
        with pytest.raises(MCSError) as ex:
            pb.set_launch_config(fpb, cap, dt)
        assert "ERR_ARG" in str(ex.value)
    assert pb.launch_config(F32)["facets_per_block"] == 2
    # a precision 1 problem has no FP64 smoother: its FP64 slot is refused
    lean = Problem(mesh.vertices, mesh.elements, mesh.lattice, 3, precision=1)
    with pytest.raises(MCSError) as ex:
        lean.set_launch_config(1, 0, F64)
    assert "ERR_ARG" in str(ex.value)
    lean.set_launch_config(2, 0, F32)
    assert lean.launch_config(F32)["facets_per_block"] == 2


@needs_lib
def test_apply_config_setter_validates():
    """mcs_set_apply_config takes 0 (the default), 1 or 2 rows of A^d per
    thread, and 4 in FP32; anything else is refused with MCS_ERR_ARG and
    leaves the choice unchanged (host only)."""
    from paper_2207_08481_amd.mcs import F32, F64, MCSError, Problem
    mesh = W.unit_cube_mesh(1)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 3)
    assert pb.apply_config(F64) == {"rows_per_thread": 0, "us_per_apply": 0.0}
    pb.set_apply_config(4, F32)
    pb.set_apply_config(1, F64)
    assert pb.apply_config(F32)["rows_per_thread"] == 4 and pb.apply_config(F64)["rows_per_thread"] == 1
    for rpt, dt in ((4, F64), (3, F32), (-1, F64), (8, F32), (1, 7)):
        with pytest.raises(MCSError) as ex:
            pb.set_apply_config(rpt, dt)
        assert "ERR_ARG" in str(ex.value)
    assert pb.apply_config(F32)["rows_per_thread"] == 4 and pb.apply_config(F64)["rows_per_thread"] == 1


def test_solve_options_setter_validates():
    """mcs_set_solve_options changes tol, max_it, inner_tol and max_outer of a
    planned problem; out-of-range values are refused with MCS_ERR_ARG (host
    only)."""
    from paper_2207_08481_amd.mcs import MCSError, Problem
    mesh = W.unit_cube_mesh(1)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 2, precision=1)
    pb.set_solve_options(0.0, 100, 0.0, 1)
    for args in ((-1.0, 10, 0.0, 1), (float("nan"), 10, 0.0, 1), (1e-8, 0, 0.0, 1), (1e-8, 10, 1.0, 1),
                 (1e-8, 10, -0.5, 1), (1e-8, 10, 1e-5, 0)):
        with pytest.raises(MCSError) as ex:
            pb.set_solve_options(*args)
        assert "ERR_ARG" in str(ex.value)


@needs_lib
def test_lowest_order_plan_and_refusals():
    """k = 1 (Sec. 7) plans in 3D with facet blocks of six dofs and no
    bubbles, also as a batch member (a group of its own) and with an outlet
    face (one more free facet layer, as for k >= 2); it is refused in 2D
    (ERR_ARG) and with the full-system variant (ERR_UNSUPPORTED)."""
    from paper_2207_08481_amd import Batch, Problem
    from paper_2207_08481_amd.mcs import MCSError
    m3 = W.unit_cube_mesh(2)
    i = Problem(m3.vertices, m3.elements, m3.lattice, 1).info
    assert (i.n_fb, i.n_bub, i.n_F, i.n_hat, i.n_p) == (6, 0, 3, 2, 1)
    m2 = W.unit_square_mesh(3)
    with pytest.raises(MCSError, match="ERR_ARG"):
        Problem(m2.vertices, m2.elements, m2.lattice, 1)
    io = Problem(m3.vertices, m3.elements, m3.lattice, 1, face_bc=[0, 1, 0, 0, 0, 0]).info
    assert io.n_fb == 6 and io.n_free_facets == i.n_free_facets + 2 * 2 * 2
    with pytest.raises(MCSError, match="ERR_UNSUPPORTED"):
        Problem(m3.vertices, m3.elements, m3.lattice, 1, smoother=2)
    b = Batch([(m3.vertices, m3.elements, m3.lattice)] * 2, [2, 1])
    assert b.info.n_groups == 2


@needs_lib
def test_batch_async_calls_need_a_started_solve():
    """mcs_batch_solve_async refuses a batch that is not bound and condensed,
    and mcs_batch_poll / mcs_batch_wait refuse when no asynchronous solve was
    started (MCS_ERR_STATE, host only)."""
    import ctypes as C
    from paper_2207_08481_amd import Batch
    from paper_2207_08481_amd.mcs import STATUS
    m3 = W.unit_cube_mesh(1)
    b = Batch([(m3.vertices, m3.elements, m3.lattice)] * 2, [2, 2])
    lib = b._lib
    state = [k for k, v in STATUS.items() if v == "ERR_STATE"][0]
    ptrs = (C.c_void_p * 2)(1, 1)
    assert lib.mcs_batch_solve_async(b._h, ptrs, ptrs) == state
    d = C.c_int32(7)
    assert lib.mcs_batch_poll(b._h, C.byref(d)) == state and d.value == 7
    assert lib.mcs_batch_wait(b._h, None) == state
    assert "no asynchronous solve" in lib.mcs_last_error().decode()
    b.close()
