"""Host-side checks of the HIP library without a GPU: it loads, exports every
symbol declared in include/stfdfd.h, validates parameters, and its partition
and local PML coefficients agree with the oracle's local operators."""
import os
import re

import numpy as np
import pytest

import workloads
from oracle import ddm, fdfd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def stf():
    import paper_2509_20801_amd as stf
    from paper_2509_20801_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libstfdfd.so not built (run python -m paper_2509_20801_amd.build)")
    _abi.load()
    return stf


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(stf_[a-z_0-9]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol(stf):
    from paper_2509_20801_amd import _abi
    lib = _abi.load()
    names = _declared_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert names <= set(_abi.EXPORTS), names - set(_abi.EXPORTS)


def _params_of(w, **over):
    p = w.params()
    d = dict(nx=p["nx"], ny=p["ny"], k0=p["k0"], dx=p["dx"], dy=p["dy"], pml=p["pml"],
             pml_order=p["pml_order"], pml_R=p["pml_R"], px=p["px"], py=p["py"],
             overlap=p["overlap"], local_pml=p["local_pml"],
             local_pml_order=p["local_pml_order"], local_pml_R=p["local_pml_R"])
    d.update(over)
    return d


@pytest.mark.parametrize("cfg", ["c1", "rand"])
def test_local_coefficients_match_oracle_local_matrix(stf, cfg):
    if cfg == "c1":
        w = workloads.configs.cylinder_tfsf()
    else:
        w = workloads.configs.small_random(nx=70, ny=57, pml=5, px=3, py=2, overlap=3, local_pml=6)
    prm = _params_of(w)
    p = w.params()
    subs = ddm.partition(p)
    gax = fdfd.global_axes(p)
    for s in subs:
        d = stf.debug_local_axes(prm, s.k)
        assert d["ox"] == s.ox and d["oy"] == s.oy and d["ix"] == s.ix and d["iy"] == s.iy
        A = ddm.local_matrix(p, w.eps_cells, s, gax).tocsr()
        nxl, nyl = s.ox[1] - s.ox[0], s.oy[1] - s.oy[0]
        idx = lambda t, u: u * nxl + t
        u0 = nyl // 2
        for t in range(1, nxl):
            assert abs(A[idx(t, u0), idx(t - 1, u0)] - d["cw"][t]) <= 1e-14 * abs(d["cw"][t])
        for t in range(nxl - 1):
            assert abs(A[idx(t, u0), idx(t + 1, u0)] - d["ce"][t]) <= 1e-14 * abs(d["ce"][t])
        t0 = nxl // 2
        for u in range(1, nyl):
            assert abs(A[idx(t0, u), idx(t0, u - 1)] - d["cs"][u]) <= 1e-14 * abs(d["cs"][u])
        for u in range(nyl - 1):
            assert abs(A[idx(t0, u), idx(t0, u + 1)] - d["cn"][u]) <= 1e-14 * abs(d["cn"][u])
        # Boundary couplings (to the Dirichlet nodes) enter the diagonal: compare
        # the diagonal minus k0^2 eps_bar.
        eb = fdfd.node_eps(w.eps_cells)[s.oy[0]:s.oy[1], s.ox[0]:s.ox[1]]
        diag = A.diagonal().reshape(nyl, nxl) - p["k0"] ** 2 * eb
        ref = -(d["cw"][None, :] + d["ce"][None, :] + d["cs"][:, None] + d["cn"][:, None])
        assert np.abs(diag - ref).max() <= 1e-13 * np.abs(ref).max()


def test_plan_statistics_c2(stf):
    prm = dict(nx=1064, ny=1064, k0=2 * np.pi / 30, pml=(20,) * 4, px=8, py=8, overlap=8,
               local_pml=16)
    info = stf.plan_query(prm)
    assert info["ndof"] == 1064 * 1064 and info["nsub"] == 64 and info["nshapes"] == 4
    # Local DoF: 172 and 176 sides.
    assert info["local_dof"] == (2 * 172 + 6 * 176) ** 2
    assert info["max_front"] <= 270
    # Nested dissection work grows like N^1.5 per subdomain: ~4.5e10 real flops.
    assert 3e10 < info["lu_flops"] < 7e10
    # Each factor entry p^2 + 2pq; O(N log N) entries per subdomain: 50-80 per local DoF.
    assert 40 < info["factor_entries"] / info["local_dof"] < 90


def test_plan_single_subdomain_counts_every_node_once(stf):
    # With one subdomain and leaf 1 x 1 boxes excluded, the dense LU of a single
    # front equal to the whole grid is the degenerate case: a leaf as large as
    # the grid gives one front with p = N, q = 0.
    prm = dict(nx=6, ny=5, k0=1.0, leaf_size=64)
    info = stf.plan_query(prm)
    assert info["nfronts"] == 1 and info["max_front"] == 30
    assert info["factor_entries"] == 30 * 30
    # LU flops of a dense 30 x 30 complex matrix: 8 * sum_{k=1}^{30} (30-k)^2.
    assert info["lu_flops"] == 8 * sum((30 - k) ** 2 for k in range(1, 31))


@pytest.mark.parametrize("bad", [dict(nx=2), dict(pml_R=1.5), dict(px=20), dict(k0=-1.0),
                                 dict(front_prec=5), dict(local_pml=0),
                                 dict(px=3, overlap=5, local_pml=12)])
def test_invalid_parameters_rejected(stf, bad):
    prm = dict(nx=132, ny=132, k0=0.3, pml=(16,) * 4, px=2, py=2, overlap=8, local_pml=16)
    prm.update(bad)
    with pytest.raises(stf.StfError) as e:
        stf.plan_query(prm)
    assert e.value.status == 1


def test_three_blocks_at_the_narrowest_width_accepted(stf):
    # 100 interior nodes in three blocks of >= 33 >= 2 (overlap + local_pml) = 32:
    # every node lies in at most two extended domains per axis.
    prm = dict(nx=132, ny=132, k0=0.3, pml=(16,) * 4, px=3, py=3, overlap=4, local_pml=12)
    assert stf.plan_query(prm)["nsub"] == 9


def test_network_parameter_count_matches_reference(stf):
    """Host-only: the library's flat parameter layout has the reference's size."""
    from oracle import nn
    for c in [nn.NNConfig(), nn.NNConfig(n=32, width=8, modes=4, layers=3),
              nn.NNConfig(n=64, width=32, modes=8, layers=2)]:
        assert stf.nn_param_count(c.n, c.width, c.modes, c.layers, c.cin) == c.nparams()
    assert stf.nn_param_count(16, 16, 9, 4) == -1          # 2M > n
    assert stf.nn_param_count(256, 12, 16, 4) == -1        # unsupported width


def test_public_header_is_plain_c(tmp_path):
    """include/stfdfd.h compiles as C99 (the ABI has no C++ types) with warnings
    as errors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "stfdfd.h"\nint main(void) { return STF_OK; }\n')
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-I", inc,
                        str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.parametrize("cfg", ["metasurface", "small", "waveguides", "disks_768", "single"])
@pytest.mark.parametrize("prec", [0, 1])
def test_launch_shape_rules_hold_on_every_level(stf, cfg, prec):
    """The built-in launch shape of every level, and every candidate the
    autotuner would time, passes the library's own validity rules (instantiated
    variant, LDS, the kernels' limits), for one and four right-hand sides."""
    p = {
        "metasurface": lambda: workloads.configs.metasurface_sheet().params(),
        "small": lambda: workloads.configs.small_random(nx=71, ny=53, pml=5, px=3, py=2, overlap=3,
                                                        local_pml=5, seed=4).params(),
        "waveguides": lambda: dict(nx=4128, ny=4128, k0=0.08, pml=(16,) * 4, px=16, py=16,
                                   overlap=8, local_pml=16),
        "disks_768": lambda: dict(nx=800, ny=800, k0=0.2, pml=(16,) * 4, px=6, py=6, overlap=8,
                                  local_pml=16),
        "single": lambda: dict(nx=200, ny=180, k0=0.3, pml=(12,) * 4, px=1, py=1),
    }[cfg]()
    for nr in (1, 4):
        levels, cands, bad = stf.debug_level_shapes(dict(p, front_prec=prec), nrhs=nr)
        assert levels >= 3 and cands >= 3 * levels and bad == 0, (levels, cands, bad)
