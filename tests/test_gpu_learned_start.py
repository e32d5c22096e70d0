"""What the trained network gains over the one-vortex start of Eq. (fun), at
small scale: the batched solver converges 128 instances of a narrow parameter
family, the U-Net trains on them on the GPU with the library's own forward
and backward kernels, and 16 held-out instances are converged from both
starts with the same kernels and criterion.  Every step is seeded and the
kernels are deterministic, so the run is reproducible."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FAMILY = dict(omega=(0.55, 0.65), g=(100.0, 200.0), nu=(1.05, 1.15))
CHANS, BOTT = (16, 32, 64, 64, 64), 64


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_06327_amd import learned_start as LS
    from paper_1906_06327_amd import nn
    return torch, LS, nn


def test_learned_start_gains(env):
    torch, LS, nn = env
    print("[learned-start] generate", flush=True)
    plist = LS.draw(128, 7, FAMILY)
    states, recs = LS.generate(plist, [13] * 128, max_steps=150000, tol=1e-6, log=print)
    X = LS._bf16_device(torch, LS.features(plist))
    T = torch.tensor(LS.make_targets(plist, states), device="cuda")
    print("[learned-start] train", flush=True)
    net = nn.UNet(8, LS.N_GRID, LS.N_GRID, chans=CHANS, bott=BOTT, seed=1)
    hist = LS.train(net, X, T, epochs=60, lr=2e-3, seed=1, log=print, log_every=0)
    print("[learned-start] loss", hist[0], "->", hist[-1], flush=True)
    assert np.isfinite(hist[-1]) and hist[-1] < 0.1 * hist[0], hist
    print("[learned-start] evaluate", flush=True)
    ev = LS.draw(16, 8, FAMILY)
    res = LS.evaluate(net.params_numpy(), ev, [13] * 16, max_steps=400000, tol=1e-7, log=print,
                      chans=CHANS, bott=BOTT)
    print(json.dumps({k: v for k, v in res.items() if k != "rows"}), flush=True)
    for r in res["rows"]:
        print(r, flush=True)
    # the learned start is much nearer to the converged lattice than Eq. (fun)
    assert res["median_distance_learned"] < 0.5 * res["median_distance_one_vortex"]
    # and it converges in fewer steps in total (an unconverged run counts its cap)
    cap = 400000
    tot0 = sum(r["steps_one_vortex"] if r["steps_one_vortex"] > 0 else cap for r in res["rows"])
    tot1 = sum(r["steps_learned"] if r["steps_learned"] > 0 else cap for r in res["rows"])
    assert tot1 < tot0, (tot1, tot0)
    assert res["same_vortex_count"] >= 12
