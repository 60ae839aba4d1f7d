"""Comparison of GPU results with the oracle, to the parity bar of the path:
|d alpha*| <= 1e-10; A_int, grad T and mdot to 1e-9 relative with absolute
floors 1e-9 h^2, 1e-9 (T range)/h and 1e-9 max|mdot|; |dn| <= 1e-9;
|dd| <= 1e-9 h; index lists and status codes exactly."""
import numpy as np

import oracle


def oracle_path(wl, **kw):
    return oracle.run_path(wl, **kw)


def check_lists(wl, gpu, eps=1e-8):
    a = wl.alpha
    mixed = np.nonzero((a > eps) & (a < 1 - eps))[0]
    band = np.nonzero(oracle.band_mask(wl.mesh, a, eps))[0]
    assert gpu["n_mixed"] == len(mixed)
    assert gpu["n_band"] == len(band)
    np.testing.assert_array_equal(gpu["mixed_idx"], mixed)
    np.testing.assert_array_equal(gpu["band_idx"], band)


def check_interface(wl, gpu, rec, h=None, report=None):
    h = h or wl.mesh.h
    idx = gpu["mixed_idx"]
    st_o = rec["status"][idx]
    st_g = gpu["status"]
    bad = np.nonzero(st_o != st_g)[0]
    msg = f"status mismatch at {len(bad)} cells, e.g. {[(int(idx[i]), int(st_o[i]), int(st_g[i])) for i in bad[:5]]}"
    assert len(bad) == 0, msg
    da = np.abs(gpu["alpha_got"] - rec["alpha_got"][idx])
    Ao = rec["A"][idx]
    dA = np.abs(gpu["A"] - Ao)
    dn = np.linalg.norm(gpu["n"] - rec["n"][:, idx], axis=0)
    dd = np.abs(gpu["d"] - rec["d"][idx])
    if report is not None:
        report.update(max_dalpha=float(da.max(initial=0)), max_dA_rel=float((dA / np.maximum(Ao, 1e-300)).max(initial=0)),
                      max_dn=float(dn.max(initial=0)), max_dd=float(dd.max(initial=0)))
    assert da.max(initial=0) <= 1e-10, f"alpha* differs by {da.max()} at cell {idx[np.argmax(da)]}"
    if len(idx) == 0:
        return
    worst = np.argmax(dA - (1e-9 * Ao + 1e-9 * h * h))
    assert np.all(dA <= 1e-9 * Ao + 1e-9 * h * h), f"A differs: cell {idx[worst]} {gpu['A'][worst]} vs {Ao[worst]}"
    assert dn.max(initial=0) <= 1e-9, f"n differs by {dn.max()} at cell {idx[np.argmax(dn)]}"
    assert dd.max(initial=0) <= 1e-9 * h, f"d differs by {dd.max()} at cell {idx[np.argmax(dd)]}"
    s_o = rec["s"][idx]
    both_nan = np.isnan(s_o) & np.isnan(gpu["s"])
    assert np.all(both_nan | (~np.isnan(s_o) & ~np.isnan(gpu["s"])))


def check_grad(wl, gpu_grad, orc_grad, cells, h=None):
    h = h or wl.mesh.h
    floor = 1e-9 * (np.ptp(wl.T) + 1e-300) / h
    g = gpu_grad[:, cells]
    o = orc_grad[:, cells]
    err = np.abs(g - o)
    tol = 1e-9 * np.abs(o) + floor
    assert np.all(err <= tol), f"grad differs: max err {err.max()} (floor {floor})"


def check_mdot(gpu_mdot, orc_mdot_at_mixed):
    floor = 1e-9 * max(np.abs(orc_mdot_at_mixed).max(initial=0), 1e-300)
    err = np.abs(gpu_mdot - orc_mdot_at_mixed)
    assert np.all(err <= 1e-9 * np.abs(orc_mdot_at_mixed) + floor), f"mdot differs: max err {err.max()}"
