"""GPU tests of how the model's table is held and exchanged: the built model stores one
column per symmetry class of the square and shares it between the offsets of that class
(checked against the oracle's independent full table elsewhere), and a table handed in from
the host (aroam_import_model: a measured or externally computed model) drives the same
kernels as a built one."""
import numpy as np
import pytest

import workloads as W
from oracle import operators as oops
from oracle import solvers as osol
from tests.helpers import oracle_supports, oracle_table, rel_l2, rel_max

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_10173_amd as P  # noqa: E402


def t64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("name", ["mid", "mid7"])
def test_built_model_stores_one_column_per_symmetry_class(name):
    cfg = W.config(name)
    g = cfg["grid"]
    K = g["k_half"]
    olo, _ = oracle_supports(name)
    a, b, k = np.nonzero(olo >= 0)
    dy, dx = np.abs(a - K), np.abs(b - K)
    classes = {(max(x, y), min(x, y), kk) for x, y, kk in zip(dx, dy, k)}
    with P.Model(cfg["sensor"], g, dtypes=("fp64", "fp32")) as m:
        info = m.info()
        H, lo, hi = m.export_table()
    assert info["n_columns"] == len(a)
    assert info["stored_columns"] == len(classes)
    assert info["stored_columns"] < info["n_columns"] / 5
    # the offsets of one class share a column exactly
    assert np.array_equal(H, H[::-1]) and np.array_equal(H, H[:, ::-1])
    assert np.array_equal(H, H.transpose(1, 0, 2, 3))
    assert rel_max(H, oracle_table(name)) <= 1e-12


def test_imported_table_reproduces_built_model():
    cfg = W.config("mid")
    g = cfg["grid"]
    x = W.random_image(cfg, 21)
    y = W.random_signal(cfg, 21)
    with P.Model(cfg["sensor"], g, dtypes=("fp64", "fp32", "bf16")) as built:
        H, lo, hi = built.export_table()
        with P.Model.from_table(g, H, lo, hi, dtypes=("fp64", "fp32", "bf16")) as imp:
            ib, ii = built.info(), imp.info()
            for key in ("n_columns", "nnz", "mac_alg", "mac_exec", "mac_exec_adj"):
                assert ib[key] == ii[key], key
            assert ii["stored_columns"] == ii["n_columns"]
            H2, lo2, hi2 = imp.export_table()
            assert np.array_equal(H2, H) and np.array_equal(lo2, lo) and np.array_equal(hi2, hi)
            for dt, conv in (("fp64", t64), ("fp32", t32), ("bf16", t32)):
                assert torch.equal(built.forward(conv(x), dt), imp.forward(conv(x), dt)), dt
                assert torch.equal(built.adjoint(conv(y), dt), imp.adjoint(conv(y), dt)), dt


def test_imported_asymmetric_table_matches_oracle():
    """A table without the sensor's symmetry (the oracle's table with a seeded factor per
    offset and a few columns cut) imported from the host: FP64 and FP32 applies and a
    Tikhonov LSQR solve match the oracle's operators on the same table."""
    name = "mid"
    cfg = W.config(name)
    g = cfg["grid"]
    K = g["k_half"]
    rng = W.rng(31)
    H = oracle_table(name) * rng.uniform(0.5, 1.5, (2 * K + 1, 2 * K + 1, 1, 1))
    H[K + 2, K - 3, :5] = 0.0                      # drop a few columns of one offset
    x = W.random_image(cfg, 22)
    y = W.random_signal(cfg, 22)
    s_ref, xa_ref = oops.forward(H, x), oops.adjoint(H, y)
    with P.Model.from_table(g, H, dtypes=("fp64", "fp32")) as m:
        H2, lo, _ = m.export_table()
        assert np.array_equal(H2, H)
        assert rel_max(m.forward(t64(x), "fp64").cpu().numpy(), s_ref) <= 1e-12
        assert rel_max(m.adjoint(t64(y), "fp64").cpu().numpy(), xa_ref) <= 1e-12
        assert rel_l2(m.forward(t32(x), "fp32").cpu().numpy(), s_ref) <= 1e-5
        assert rel_l2(m.adjoint(t32(y), "fp32").cpu().numpy(), xa_ref) <= 1e-5
        assert m.info()["n_elements"] == 0
        shp_x, shp_s = x.shape, y.shape
        A = lambda v: oops.forward(H, v.reshape(shp_x)).ravel()
        AT = lambda u: oops.adjoint(H, u.reshape(shp_s)).ravel()
        s = A(W.make_phantom(cfg, 0).ravel())
        lam = osol.lam_l2(AT(s))
        x_ref, _ = osol.lsqr(A, AT, s, damp=np.sqrt(lam), iters=20)
        xg, info = m.solve_lsqr(t64(s.reshape(shp_s)), lam=-1.0, iters=20, inner="fp64")
        assert abs(info["lam"] - lam) <= 1e-12 * lam
        assert rel_l2(xg.cpu().numpy(), x_ref) <= 1e-10


def test_repeated_applies_and_solves_hold_device_memory_steady():
    """Single applies and solves take their temporaries (stage buffers with partial slots,
    solver vectors) from the library's memory pool, which keeps freed blocks: after a first
    round, further rounds of the same calls allocate nothing more from the device."""
    name = "mid"
    cfg = W.config(name)
    g = cfg["grid"]
    x = t32(W.random_image(cfg, 31))
    y = t32(W.random_signal(cfg, 31))
    with P.Model(cfg["sensor"], g, dtypes=("fp32", "bf16", "fp8")) as m:
        def rounds(n):
            for _ in range(n):
                for dt in ("fp32", "bf16", "fp8"):
                    m.forward(x, dt)
                    m.adjoint(y, dt)
                m.solve_lsqr(y, lam=-1.0, iters=5, inner="bf16", outer="fp32", refine_sweeps=1)
                m.solve_l1(y, lam=-1.0, iters=5, inner="fp32")
            torch.cuda.synchronize()
        rounds(2)
        free0 = torch.cuda.mem_get_info()[0]
        rounds(10)
        free1 = torch.cuda.mem_get_info()[0]
    print(f"[memory] free before {free0 / 2**20:.0f} MiB, after {free1 / 2**20:.0f} MiB")
    assert free0 - free1 <= 16 << 20
