"""The surrogate's bf16 matrix-core kernels against the float64 reference that
reproduces their rounding points (oracle.surrogate)."""
import numpy as np
import pytest
import torch

from oracle import surrogate as S
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(0, 1, (n, 6)), rng.uniform(-4, 4, (n, 1)),
                        rng.uniform(0.05, 3, (n, 1))], axis=1).astype(np.float32)
    t = rng.uniform(0, 1, n).astype(np.float32)
    return x, t


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 70001])
def test_mlp_forward_matches_reference(n):
    from paper_2512_11800_amd import surrogate as G
    theta = S.init_params(1).astype(np.float32)
    x, _ = _batch(n, 2)
    packed = G.mlp_pack(torch.tensor(theta, device="cuda"))
    f = G.mlp_forward(packed, torch.tensor(x, device="cuda")).cpu().numpy()
    ref, _ = S.forward(theta.astype(np.float64), x.astype(np.float64))
    e = np.abs(f - ref)
    err = e.max()
    frac = float((e > 1e-4).mean())
    log(f"[mlp] forward n={n} max|F - ref| = {err:.3e} median={np.median(e):.1e} frac>1e-4={frac:.1e}")
    # float32 (GPU) and float64 (reference) activations can round to
    # neighbouring bf16 values at ties: one such flip moves F by <~1e-3
    assert np.median(e) < 1e-6
    assert frac < 1e-3
    assert err < 2e-3


def test_mlp_loss_grad_matches_reference():
    from paper_2512_11800_amd import surrogate as G
    theta = S.init_params(3).astype(np.float32)
    x, t = _batch(5000, 4)
    packed = G.mlp_pack(torch.tensor(theta, device="cuda"))
    loss, grad = G.mlp_loss_grad(packed, torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"))
    loss, grad = float(loss.item()), grad.cpu().numpy().astype(np.float64)
    lref, gref = S.loss_grad(theta.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    log(f"[mlp] loss gpu={loss:.6e} ref={lref:.6e}")
    assert loss == pytest.approx(lref, rel=1e-4)
    o = 0
    for k, s in S.SIZES.items():
        m = int(np.prod(s))
        a, b = grad[o:o + m], gref[o:o + m]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        log(f"[mlp] grad {k}: rel_err={rel:.3e}")
        assert rel < 3e-3, k
        o += m


def test_adam_step_matches_reference():
    from paper_2512_11800_amd import surrogate as G
    rng = np.random.default_rng(5)
    p = rng.normal(size=S.N_PARAMS).astype(np.float32)
    g = rng.normal(size=S.N_PARAMS).astype(np.float32)
    m = rng.normal(size=S.N_PARAMS).astype(np.float32) * 0.1
    v = np.abs(rng.normal(size=S.N_PARAMS).astype(np.float32)) * 0.1
    tp, tm, tv = (torch.tensor(a, device="cuda") for a in (p, m, v))
    G.adam_step(tp, tm, tv, torch.tensor(g, device="cuda"), 7, 1e-3)
    rp, rm, rv = S.adam(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                        g.astype(np.float64), 7, 1e-3)
    assert np.allclose(tp.cpu().numpy(), rp, rtol=1e-5, atol=1e-7)
    assert np.allclose(tm.cpu().numpy(), rm, rtol=1e-5, atol=1e-7)
    assert np.allclose(tv.cpu().numpy(), rv, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss():
    """A few hundred steps on a smooth synthetic target learn it."""
    from paper_2512_11800_amd import surrogate as G
    rng = np.random.default_rng(6)
    n = 200_000
    x = np.concatenate([rng.normal(0, 1, (n, 6)), rng.uniform(-4, 4, (n, 1)),
                        rng.uniform(0.1, 3, (n, 1))], axis=1).astype(np.float32)
    f_true = 1 / (1 + np.exp(-(1.5 * x[:, 6] + 0.3 * x[:, 0])))
    t = np.exp(-x[:, 7] * f_true).astype(np.float32)
    xt, tt = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    theta, packed, losses = G.train(xt, tt, steps=300, batch=8192, lr=3e-3, log_every=50)
    log(f"[mlp] training losses {losses}")
    assert losses[-1][1] < 0.1 * losses[0][1]
