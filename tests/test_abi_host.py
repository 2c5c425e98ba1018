"""CPU-side checks of the C ABI library: it loads, exports every declared entry
point, validates arguments, and its host set-up tables (written independently
in C++) agree with the oracle.  No device call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1910_11505_amd as sg
from paper_1910_11505_amd.binding import make_problem
from oracle import kl as okl
from oracle import pc as opc
from oracle.precond import make_groups
from oracle.system import SGSystem
from synth import CONFIGS, Problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sg.h")).read()
    return sorted(set(re.findall(r"\b(sg_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = sg.load_library()
    names = _declared()
    assert "sg_apply" in names and "sg_gmres_solve" in names
    for name in names:
        assert hasattr(lib, name), name


def _setup(**kw):
    base = dict(n=16, M=2, p=2, q=4, cov="exp_l1", mu=0.0, sigma=0.5, corr_len=0.5, a_min=0.01)
    base.update(kw)
    return sg.sg_setup(make_problem(**base))


@pytest.mark.parametrize("kw", [dict(n=12), dict(n=2), dict(M=0), dict(p=-1), dict(q=17),
                                dict(sigma=-1.0), dict(corr_len=0.0), dict(a_min=-0.1),
                                dict(cov=7), dict(sigma=float("nan"))])
def test_invalid_problem_rejected(kw):
    with pytest.raises(sg.SGError) as e:
        _setup(**kw)
    assert e.value.code == -1


def test_unsupported_size_rejected():
    with pytest.raises(sg.SGError) as e:
        _setup(M=6, p=6, q=6)          # P = 924 modes
    assert e.value.code == -2


def test_device_calls_need_binding():
    h = _setup()
    with pytest.raises(sg.SGError) as e:
        sg.sg_apply(h, 256, 512, 0)
    assert e.value.code == -4
    with pytest.raises(sg.SGError):
        sg.sg_precond_apply(h, "mean", "klvar", 256, 256, 0)   # aliasing / not bound
    sg.sg_destroy(h)


def test_new_entry_points_validate_before_any_device_call():
    """The full-system multigrid, the stage objective, the network's backward
    pass and its Adam state check their arguments (and the handle's binding)
    before touching the device."""
    lib = sg.load_library()
    h = _setup()
    assert sg.sg_mg_workspace_bytes(h, 7) == 0                   # unknown grouping
    assert sg.sg_mg_workspace_bytes(h, "all") > 0
    with pytest.raises(sg.SGError) as e:
        sg.sg_mg_bind(h, "fg", 256, 1 << 20, 0)                # handle not bound
    assert e.value.code == -4
    assert lib.sg_cnn_stage_work_doubles(None) == 0
    assert sg.sg_cnn_stage_work_doubles(h) > 5 * 6 * 15 * 15
    # null network / workspace, then an unbound handle
    assert lib.sg_cnn_stage_grad(h, None, 256, 0, 0, 1, 256, None, None) == -1
    assert lib.sg_cnn_stage_grad(h, 512, 256, 0, 0, 1, None, None, None) == -1
    assert lib.sg_cnn_backward(None, 1, 0, ctypes.c_float(0.0), 1, None) == -1
    assert lib.sg_cnn_get_adam(None, None, None, None, None) == -1
    assert lib.sg_cnn_set_adam(None, None, None, None, None, None) == -1
    sg.sg_destroy(h)


def test_nonfinite_forcing_rejected():
    f = np.ones(17 * 17)
    f[5] = np.inf
    with pytest.raises(sg.SGError) as e:
        sg.sg_setup(make_problem(16, 2, 2, 4), f)
    assert e.value.code == -1


@pytest.mark.parametrize("M,p,q", [(2, 2, 4), (4, 3, 6), (6, 3, 6), (3, 2, 3)])
def test_sizes_match_oracle(M, p, q):
    h = _setup(M=M, p=p, q=q)
    P, Nh, na, nnz = sg.sg_sizes(h)
    Jp, Jq = opc.multi_indices(M, p), opc.multi_indices(M, q)
    assert (P, Nh, na, nnz) == (len(Jp), 15 * 15, len(Jq), len(opc.triple_products(Jp, Jq)[3]))
    assert sg.sg_workspace_bytes(h) > 8 * na * 4 * 16 * 16
    sg.sg_destroy(h)


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_kl_tables_match_oracle(name):
    pr = CONFIGS[name]
    h = _setup(n=pr.n, M=pr.M, p=pr.p, q=pr.q, cov=pr.cov, sigma=pr.sigma, corr_len=pr.corr_len)
    lam = np.zeros(pr.M)
    sg.sg_export(h, "kl", 0, lam)
    gq = np.zeros(pr.M * 4 * pr.n * pr.n)
    sg.sg_export(h, "gq", 0, gq)
    olam, B, _ = okl.kl_2d(pr.n, pr.cov, pr.corr_len, pr.sigma, pr.M)
    og = okl.g_at_quad(pr.n, olam, B).reshape(-1)
    assert np.allclose(lam, olam, rtol=1e-12, atol=0)
    assert np.abs(gq - og).max() <= 1e-12 * np.abs(og).max()
    sg.sg_destroy(h)


@pytest.mark.parametrize("M,p", [(2, 4), (4, 3), (6, 3), (3, 3)])
@pytest.mark.parametrize("gname,gid", [("klvar", 0), ("klvar_meansep", 1), ("permode", 2), ("fg", 3),
                                         ("all", 4)])
def test_groupings_match_oracle(M, p, gname, gid):
    h = _setup(M=M, p=p, q=2 * p)
    out = np.zeros(2000)
    sg.sg_export(h, "groups", gid, out)
    S = int(out[0])
    pos, got = 1, []
    for _ in range(S):
        sz = int(out[pos])
        got.append([int(v) for v in out[pos + 1:pos + 1 + sz]])
        pos += 1 + sz
    assert got == make_groups(opc.multi_indices(M, p), gname)
    sg.sg_destroy(h)


def test_set_apply_validation():
    h = _setup()                                   # q = 2p: both forms available
    sg.sg_set_apply(h, "factored", 16, stream=0)
    sg.sg_set_apply(h, "triple", 0, stream=0)
    sg.sg_set_apply(h, "auto", 0, stream=0)
    for bad_kind, bad_qb in ((3, 0), (-1, 0), (0, 12), (2, 128)):
        with pytest.raises(sg.SGError) as e:
            sg.sg_set_apply(h, bad_kind, bad_qb, stream=0)
        assert e.value.code == -1
    sg.sg_destroy(h)
    h = _setup(M=3, p=2, q=3)                      # q < 2p: factored form is not exact
    with pytest.raises(sg.SGError) as e:
        sg.sg_set_apply(h, "factored", 0, stream=0)
    assert e.value.code == -2
    sg.sg_set_apply(h, "triple", 0, stream=0)
    sg.sg_destroy(h)


def test_set_apply_oversized_batch_keeps_plan():
    h = _setup(M=6, p=4, q=8, n=8)                 # P = 210: 64 points need > 160 KB of LDS
    with pytest.raises(sg.SGError) as e:
        sg.sg_set_apply(h, "factored", 64, stream=0)
    assert e.value.code == -2
    sg.sg_set_apply(h, "factored", 8, stream=0)
    sg.sg_destroy(h)


def test_q2_setup_validates_and_reports_refined_sizes():
    """sg_setup_q2: n2 elements per side give (2 n2 - 1)^2 unknowns per mode;
    the factored-only apply rejects q < 2p; the form query reports 3 and the
    form setter refuses (no device call is made)."""
    base = dict(n=8, M=2, p=2, q=4, cov="exp_l1", mu=0.0, sigma=0.5, corr_len=0.5, a_min=0.01)
    h = sg.sg_setup_q2(make_problem(**base))
    P, Nh, _, _ = sg.sg_sizes(h)
    assert (P, Nh) == (6, 15 * 15)
    assert sg.sg_apply_form(h)[0] == 3
    with pytest.raises(sg.SGError) as e:
        sg.sg_set_apply(h, 2, 0, 0)
    assert e.value.code == -2
    sg.sg_destroy(h)
    for kw, code in ((dict(q=3), -2), (dict(n=6), -1), (dict(n=4096), -1)):
        with pytest.raises(sg.SGError) as e:
            sg.sg_setup_q2(make_problem(**{**base, **kw}))
        assert e.value.code == code
