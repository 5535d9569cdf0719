"""Comparison of HIP-path outputs with the FP64 oracle (shared test helper).

Bars (float32 path):
  labels  equal for every query the oracle does not mark ambiguous; counts in
          [count_lo, count_hi]; neighbourhood sizes in [nbr_lo, nbr_hi]
  min     |gpu - oracle| <= 1e-5 max(|oracle|, tstar)
  softmin |gpu - oracle| <= 1e-5 max(|oracle|, tsoft) + 1e-5 tau
  cost    the sums (cost * |N|) agree to 1e-5 max(1, gamma tcost) relative
          (plus the contribution of ball-boundary pairs when |N| differs)
tstar/tsoft/tcost are the un-cancelled magnitudes T = s^2 + n sqrt(sigma^2)
of the pairs that decide each result (see the oracle).
"""
import numpy as np

RTOL = 1e-5


def compare(gpu: dict, ref: dict, tau: float, gamma: float, d_max: float = 1.0, rtol: float = RTOL,
            where: str = ""):
    stats = {}
    amb = ref["ambiguous"].astype(bool)
    if "label" in gpu:
        lab = np.asarray(gpu["label"])
        bad = (lab != ref["label"]) & ~amb
        assert not bad.any(), f"{where}: {bad.sum()} label mismatches at {np.argwhere(bad)[:5].tolist()}"
        stats["label_flips_ambiguous"] = int(((lab != ref["label"]) & amb).sum())
    if "count" in gpu:
        c = np.asarray(gpu["count"])
        lo, hi = ref["count_lo"], ref["count_hi"]
        bad = (c < lo) | (c > hi)
        assert not bad.any(), (f"{where}: {bad.sum()} counts outside the band, e.g. "
                               f"{[(int(c[i]), int(lo[i]), int(hi[i])) for i in map(tuple, np.argwhere(bad)[:5])]}")
        stats["count_exact"] = float((c == ref["count"]).mean())
    if "nbr" in gpu:
        nb = np.asarray(gpu["nbr"]).astype(np.int64)
        bad = (nb < ref["nbr_lo"]) | (nb > ref["nbr_hi"])
        assert not bad.any(), f"{where}: {bad.sum()} neighbourhood sizes outside the band"
    if "min" in gpu:
        g, o = np.asarray(gpu["min"], np.float64), ref["min"]
        inf = np.isinf(o)
        assert np.array_equal(np.isinf(g), inf), f"{where}: min infinities differ"
        err = np.abs(g[~inf] - o[~inf])
        tol = rtol * np.maximum(np.abs(o[~inf]), ref["tstar"][~inf])
        assert np.all(err <= tol), f"{where}: min err {np.max(err / tol):.3g} x tol"
        stats["min_max_rel"] = float(np.max(err / np.maximum(np.abs(o[~inf]), ref["tstar"][~inf]), initial=0))
    if "softmin" in gpu:
        g, o = np.asarray(gpu["softmin"], np.float64), ref["softmin"]
        inf = np.isinf(o)
        assert np.array_equal(np.isinf(g), inf), f"{where}: softmin infinities differ"
        err = np.abs(g[~inf] - o[~inf])
        tol = rtol * np.maximum(np.abs(o[~inf]), ref["tsoft"][~inf]) + rtol * tau
        assert np.all(err <= tol), f"{where}: softmin err {np.max(err / tol):.3g} x tol"
        stats["softmin_max_rel"] = float(np.max(err / (tol / rtol), initial=0))
    if "cost" in gpu:
        g, o = np.asarray(gpu["cost"], np.float64), ref["cost"]
        nb_g = (np.asarray(gpu["nbr"], np.float64) if "nbr" in gpu else ref["nbr"].astype(np.float64))[:, None]
        nb_o = ref["nbr"].astype(np.float64)[:, None]
        sg, so = g * nb_g, o * nb_o
        # pairs on the ball boundary contribute at most d_max exp(-gamma (s~^2 - 1)) each;
        # bound that by d_max per differing pair times their tiny weight via the band size
        extra = np.abs(nb_g - nb_o) * d_max
        tol = rtol * np.abs(so) * np.maximum(1.0, gamma * ref["tcost"]) + 1e-30 * d_max + extra
        err = np.abs(sg - so)
        assert np.all(err <= tol), f"{where}: cost err {np.max(err / tol):.3g} x tol"
        nz = so > 1e-30
        stats["cost_max_rel"] = float(np.max(err[nz] / so[nz], initial=0))
    return stats
