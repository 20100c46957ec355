"""The FWI loop (paper_2009_12623_amd.fwi) on a small 2D survey: the
objective decreases, the model changes only where the mask allows, and the run with
compressed checkpoints follows the exact run's trajectory closely (Sec. 4
"Convergence")."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

F = pytest.importorskip("paper_2009_12623_amd.fwigrad")
from paper_2009_12623_amd import fwi  # noqa: E402

DEV = "cuda:0"


def survey():
    base = synth.tiny_shot(2, n=60, so=8, nbl=10, nt=260)
    v0, vt = synth.tiny_models(base.shape, seed=11)
    shots = [synth.Shot(2, base.shape, base.h, base.so, base.nbl, base.nt, base.dt, base.vmax, base.f0,
                        (x, 2), base.rec) for x in (10, 30, 50)]
    tomt = lambda v: torch.from_numpy(synth.slowness2(synth.extend(v, base.nbl)).astype(np.float32)).to(DEV)
    q = torch.from_numpy(base.wavelet().astype(np.float32)).to(DEV)
    mask = torch.zeros(base.comp_shape, device=DEV)
    nbl = base.nbl
    mask[nbl:-nbl, nbl + 5:-nbl] = 1.0
    return shots, tomt(v0), tomt(vt), q, mask


def test_fwi_decreases_and_compressed_follows_exact():
    c = F.Context(0, pool_bytes=1 << 28)
    shots, m0, mt, q, mask = survey()
    d_obs = [c.forward(s, mt, q) for s in shots]
    ex = fwi.run_fwi(c, shots, m0, q, d_obs, iterations=6, nslots=20, compress=False, step=0.05,
                     vmin=1400.0, vmax=2600.0, mask=mask)
    lo = fwi.run_fwi(c, shots, m0, q, d_obs, iterations=6, nslots=20, compress=True, atol=1e-3,
                     step=0.05, vmin=1400.0, vmax=2600.0, mask=mask)
    pe, pl = np.array(ex["objective"]), np.array(lo["objective"])
    print("exact", pe, "lossy", pl)
    assert pe[-1] < 0.7 * pe[0]
    assert np.all(np.diff(pe) < 0)
    assert np.max(np.abs(pl - pe) / pe) < 1e-2
    # the update stays inside the mask
    assert torch.equal(ex["m"][mask == 0], m0[mask == 0])
    assert not torch.equal(ex["m"][mask == 1], m0[mask == 1])
    c.close()


def test_fwi_iterations_match_the_oracle_loop():
    """three iterations of the GPU loop (exact checkpoints) against the FP64
    oracle loop (oracle/fwi.py, the same reading of the step rule written
    independently): objective before each iteration and after the last, and
    the final model update; every line-search decision of the oracle run
    clears its threshold by a wide margin, so both runs take the same ones"""
    from oracle import fwi as ofwi
    from oracle import solver
    c = F.Context(0, pool_bytes=1 << 28)
    shots, m0, mt, q, mask = survey()
    qh = q.double().cpu().numpy()
    mth = mt.double().cpu().numpy()
    d_obs_h = [solver.forward(solver.Problem(s, mth, wavelet=qh)) for s in shots]
    d_obs = [torch.from_numpy(d.astype(np.float32)).to(DEV) for d in d_obs_h]
    ref = ofwi.run_fwi(shots, m0.double().cpu().numpy(), qh, d_obs_h, 3, 0.05, 1400.0, 2600.0,
                       mask.double().cpu().numpy())
    print("oracle objective", ref["objective"], "decreases", ref["decreases"])
    assert min(abs(x) for x in ref["decreases"]) > 1e-3
    run = fwi.run_fwi(c, shots, m0, q, d_obs, iterations=3, nslots=20, compress=False, step=0.05,
                      vmin=1400.0, vmax=2600.0, mask=mask)
    po, pr = np.array(run["objective"]), np.array(ref["objective"])
    print("gpu objective", po)
    assert np.max(np.abs(po - pr) / pr) <= 1e-4
    m0h = m0.double().cpu().numpy()
    upd_g = run["m"].double().cpu().numpy() - m0h
    upd_o = ref["m"] - m0h
    err = np.linalg.norm(upd_g - upd_o) / np.linalg.norm(upd_o)
    print("model update rel L2 %.2e" % err)
    assert err <= 1e-4
    c.close()
