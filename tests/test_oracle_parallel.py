"""The process-parallel drivers of the oracle (oracle.parallel) reproduce the serial oracle:
PI tables and reconstruction bit for bit, and the adjoint rows of single views equal the
rows of the whole transpose recon_T."""
import numpy as np

import oracle as O
from oracle import parallel as OP
from synth import configs, phantom


def _case():
    wl = configs.with_helix_offsets(configs.tiny(nxy=14, nz=30, cols=48, rows=8, views_per_turn=72,
                                                 turns=5, feed=24.0, dxy=2.0, slices_per_pitch=12))
    geom, gr = wl.geom.as_dict(), wl.grid.as_dict()
    ph = phantom.make_phantom(wl.phantom, gr, wl.seed)
    return geom, gr, phantom.project(ph, geom).astype(np.float32)


def test_parallel_tables_and_recon_equal_serial():
    geom, gr, g = _case()
    scan = O.Scan(geom)
    tab0 = O.pitch_tables(scan, gr)
    tab1 = OP.pitch_tables(geom, gr, workers=3)
    for k in ("lam_i", "lam_o", "li", "lo", "nf", "nl", "fov", "n_lo", "n_hi"):
        assert np.array_equal(tab0[k], tab1[k]), k
    f0, v0 = O.recon(scan, gr, g, tables=tab0)
    f1, v1 = OP.recon(geom, gr, g, workers=3, tables=tab1)
    assert np.array_equal(v0, v1) and v0.sum() > 1000
    assert np.array_equal(f0, f1)


def test_adjoint_rows_equal_the_whole_transpose():
    geom, gr, _ = _case()
    scan = O.Scan(geom)
    fbar = np.random.default_rng(3).normal(size=(gr["nz"], gr["ny"], gr["nx"]))
    whole = O.recon_T(scan, gr, fbar)
    views = [1, 100, 150, 200, 250, 358]
    rows = OP.adjoint_views(geom, gr, fbar, views, workers=3)
    for n in views:
        assert np.abs(rows[n] - whole[n]).max() <= 1e-12 * np.abs(whole).max(), n
    assert all(np.abs(rows[n]).max() > 0 for n in views[1:-1])
