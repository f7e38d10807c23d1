"""GPU parity of the score and probability-flow pass (xkp_score_flow) against the oracle on
ragged sizes, both fields, with and without drift and with skipped outputs; the embedding of a
whole chain against the oracle's chain.  Every call goes through the C ABI."""
import numpy as np
import pytest

from gpu_util import cpu, dev, t64
from oracle import epilogue as E

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


@pytest.mark.parametrize("field", ["mt", "x"])
def test_score_flow_matches_oracle(X, field):
    import torch
    Hs = [5, 31, 64, 100, 17]          # n = 25 .. 10000: partial blocks and odd sides
    rng = np.random.default_rng(11)
    ctx = X.Context(max(Hs) ** 2, 8, len(Hs))
    specs, data = [], []
    for k, H in enumerate(Hs):
        n = H * H
        mt, xs = rng.normal(size=n), rng.normal(size=n)
        fx = rng.normal(size=n) if k % 2 else None
        fy = rng.normal(size=n) if k % 2 else None
        dt, g = 1.0 / (10 + k), 0.3 + 0.1 * k
        tens = dict(mt=t64(mt), x=t64(xs), b=torch.zeros(n, dtype=torch.float64, device=dev()),
                    fx=None if fx is None else t64(fx), fy=None if fy is None else t64(fy))
        specs.append(X.SystemSpec(H, dt, g, tens["mt"], b=tens["b"], x=tens["x"],
                                  fx=tens["fx"], fy=tens["fy"]))
        data.append((H, mt if field == "mt" else xs, g, dt, fx, fy))
    d = X.pack_systems(specs, dev())
    score = [torch.full((2 * H * H,), 7.0, dtype=torch.float64, device=dev()) for H in Hs]
    d0 = [rng.normal(size=2 * H * H) for H in Hs]
    disp = [t64(v) for v in d0]
    sp = torch.tensor([t.data_ptr() for t in score], dtype=torch.int64, device=dev())
    dp = torch.tensor([t.data_ptr() for t in disp], dtype=torch.int64, device=dev())
    # the third system's score is not wanted (NULL entry)
    sp[2] = 0
    fid = X.FIELD_MT if field == "mt" else X.FIELD_X
    ctx.score_flow(d, len(Hs), fid, sp, dp)
    torch.cuda.synchronize()
    for k, (H, m, g, dt, fx, fy) in enumerate(data):
        sx, sy = E.score(H, m)
        ref_s = np.concatenate([sx, sy])
        got_s = cpu(score[k])
        if k == 2:
            assert np.all(got_s == 7.0)
        else:
            assert np.abs(got_s - ref_s).max() <= 1e-14 * np.abs(ref_s).max(), H
        ref_d = E.flow_step(d0[k], H, m, g, dt, fx, fy).reshape(-1)
        assert np.abs(cpu(disp[k]) - ref_d).max() <= 1e-14 * np.abs(ref_d).max(), H
    # score only (no displacement array), then host argument errors
    ctx.score_flow(d, len(Hs), fid, sp, None)
    torch.cuda.synchronize()
    with pytest.raises(X.XkpError):
        ctx.score_flow(d, len(Hs), 2, sp, dp)


def test_chain_embedding_matches_oracle(X):
    """28x28 workload (1 seed + 1 target, T = 50): the displacement after the whole chain, one
    flow step per timestep from the state before the step, against the oracle chain's."""
    import torch
    from oracle.chain import run_chain
    from paper_2511_17634_amd.driver import Chain
    from synth import CONFIGS, config_images, initial_state
    cfg = CONFIGS["c1"]
    H = cfg.groups[0].H
    seed, tg = config_images(cfg, 0, 0, 1)
    s0, t0 = initial_state(seed[0]), initial_state(tg[0, 0])[None]
    ch = Chain(H, cfg.T, cfg.m, s0, t0, embed=True)
    ch.run()
    torch.cuda.synchronize()
    disp = np.zeros((2, H * H))
    last = {}

    def on_step(n, ms, mt):
        nonlocal disp
        disp = E.flow_step(disp, H, mt[0], cfg.g, 1.0 / cfg.T)
        last["m"] = mt[0].copy()

    run_chain(s0, t0, H, cfg.T, cfg.m, on_step=on_step)
    got = cpu(ch.disp_t[0])
    # each state agrees to about T tol |m|; the displacement sums T scores of them
    assert np.abs(got - disp).max() <= 1e-5 * np.abs(disp).max()
    sx, sy = E.score(H, last["m"])
    ref = np.stack([sx, sy])
    assert np.abs(cpu(ch.score_t[0]) - ref).max() <= 1e-5 * np.abs(ref).max()
    # a second run starts from a zero displacement again
    ch.run()
    torch.cuda.synchronize()
    assert np.abs(cpu(ch.disp_t[0]) - got).max() <= 1e-12 * np.abs(got).max()
