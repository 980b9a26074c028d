"""GPU parity of the differentiable energy: gpr_energy_forces_dev / gpr_energy_backward_dev
(through the C ABI and through the torch.autograd binding) against the FP64 oracle's forces and
parameter gradient, itself pinned by closed forms and central finite differences.  Bar: 1e-4 of
the largest component, per parameter kind, relative; energies 1e-5 relative."""
import sys

import numpy as np
import pytest

import gpr_synth as G
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    return torch


def _oracle_weighted(spec, X, w):
    o = oracle.System(dict(spec, n_replicas=2))
    tot = None
    for r in range(len(w)):
        g = o.param_grad(X[r])
        if tot is None:
            tot = {k: w[r] * v for k, v in g.items()}
        else:
            for k in tot:
                tot[k] = tot[k] + w[r] * g[k]
    return tot


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-30)


def _positions(spec, steps):
    """float32 positions of every replica after some stepping (replicas differ by their noise)."""
    import paper_1807_02431_amd as gpr
    g = gpr.System(spec)
    g.advance(steps)
    return np.stack([g.get_state(r)[0] for r in range(spec["n_replicas"])]).astype(np.float32)


@pytest.mark.parametrize("name,R,steps", [("chain22", 4, 300), ("rl300", 4, 40), ("rl2432", 64, 20)])
def test_backward_matches_oracle(name, R, steps):
    import paper_1807_02431_amd as gpr
    torch = _torch()
    spec = G.round_to_f32(G.config(name, n_replicas=R))
    say("backward", name, R)
    X = _positions(spec, steps)
    s = gpr.System(spec, stream=torch.cuda.current_stream())
    x = torch.tensor(X, device="cuda")
    U = torch.empty(R, dtype=torch.float64, device="cuda")
    F = torch.empty_like(x)
    s.energy_forces_dev(x.data_ptr(), U.data_ptr(), F.data_ptr())
    w = torch.tensor(np.random.default_rng(7).normal(size=R), dtype=torch.float64, device="cuda")
    dx = torch.empty_like(x)
    n, nt = s.n, s.nt
    ge, gs, gq = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3))
    gk = torch.empty(max(1, nt), dtype=torch.float64, device="cuda")
    s.energy_backward_dev(w.data_ptr(), dx.data_ptr(), ge.data_ptr(), gs.data_ptr(), gq.data_ptr(), gk.data_ptr())
    wn = w.cpu().numpy()
    o = oracle.System(dict(spec, n_replicas=2))
    for r in range(0, R, max(1, R // 8)):
        Uo, Fo = o.eval(X[r])
        assert abs(U[r].item() - Uo) <= 1e-5 * abs(Uo)
        assert _rel(F[r].cpu().numpy(), Fo) < 1e-5
        assert _rel(dx[r].cpu().numpy(), -wn[r] * Fo) < 1e-5
    ref = _oracle_weighted(spec, X, wn)
    for key, got in (("epsilon", ge), ("sigma", gs), ("charge", gq), ("torsion_k", gk[:nt])):
        err = _rel(got.cpu().numpy(), ref[key])
        say(key, "rel err", err)
        assert err < 1e-4, key


def test_autograd_energy_model():
    """torch.autograd over the library: gradients of sum_r w_r U_r with respect to positions and
    parameters, a parameter change taking effect in the next forward pass, and a backward pass
    after a later forward pass (the earlier positions are put back)."""
    torch = _torch()
    from paper_1807_02431_amd.autograd import EnergyModel
    spec = G.round_to_f32(G.config("rl300", n_replicas=4))
    X = _positions(spec, 30)
    model = EnergyModel(spec)
    eps, sig, chg, tk = (t.requires_grad_() for t in model.parameters())
    x = torch.tensor(X, device="cuda", requires_grad=True)
    w = torch.tensor([0.5, -1.0, 2.0, 0.25], dtype=torch.float64, device="cuda")
    U = model(x, eps, sig, chg, tk)
    # a second evaluation at other positions before the first backward
    x2 = torch.tensor(X[::-1].copy(), device="cuda")
    model(x2, eps.detach(), sig.detach(), chg.detach(), tk.detach())
    (w * U).sum().backward()
    wn = w.cpu().numpy()
    o = oracle.System(dict(spec, n_replicas=2))
    for r in range(4):
        Uo, Fo = o.eval(X[r])
        assert abs(U[r].item() - Uo) <= 1e-5 * abs(Uo)
        assert _rel(x.grad[r].cpu().numpy(), -wn[r] * Fo) < 1e-5
    ref = _oracle_weighted(spec, X, wn)
    for key, t in (("epsilon", eps), ("sigma", sig), ("charge", chg), ("torsion_k", tk)):
        assert _rel(t.grad.cpu().numpy(), ref[key]) < 1e-4, key
    # new parameters: the energy follows the oracle with the same parameters
    eps2 = (eps.detach() * 1.1).requires_grad_()
    U2 = model(x, eps2, sig.detach(), chg.detach(), tk.detach())
    spec2 = dict(spec, epsilon=np.asarray(spec["epsilon"]) * 1.1)
    o2 = oracle.System(dict(spec2, n_replicas=2))
    for r in range(4):
        assert abs(U2[r].item() - o2.eval(X[r])[0]) <= 1e-5 * abs(o2.eval(X[r])[0])
    U2.sum().backward()
    ref2 = _oracle_weighted(spec2, X, np.ones(4))
    assert _rel(eps2.grad.cpu().numpy(), ref2["epsilon"]) < 1e-4


def test_parameters_change_the_dynamics_consistently():
    """gpr_set_params between stepping calls: the forces the integrator carries are those of
    the new parameters (compared with the oracle at the same positions)."""
    import paper_1807_02431_amd as gpr
    spec = G.round_to_f32(G.config("rl300", n_replicas=2))
    g = gpr.System(spec, path=gpr.PATH_PERSISTENT)
    g.advance(10)
    chg = np.asarray(spec["charge"]) * 0.5
    tk = np.asarray(spec["torsion_k"]) * 2.0
    g.set_params(charge=chg, torsion_k=tk)
    E, F = g.energy_forces()
    o = oracle.System(dict(spec, charge=chg, torsion_k=tk))
    for r in range(2):
        q, _ = g.get_state(r)
        Uo, Fo = o.eval(q)
        assert _rel(F[r], Fo) < 1e-5
    g.advance(10)
    with pytest.raises(gpr.GprError):
        g.set_params(epsilon=-np.ones(spec["n_atoms"]))


def test_backward_of_an_earlier_pass_uses_its_own_parameters():
    """forward(p1), forward(p2), then the backward of the first pass: its gradients are those
    of p1 at the first pass's positions (oracle gradient at p1), not of the later p2."""
    import torch
    from paper_1807_02431_amd.autograd import EnergyModel
    spec = G.round_to_f32(G.config("rl300", n_replicas=4))
    model = EnergyModel(spec)
    eps, sig, chg, tk = [t.requires_grad_() for t in model.parameters()]
    X = np.stack([np.asarray(spec["pos"], np.float32)] * 4)
    X[1:] += np.random.default_rng(3).normal(scale=0.01, size=X[1:].shape).astype(np.float32)
    x1 = torch.tensor(X, device="cuda", requires_grad=True)
    U1 = model(x1, eps, sig, chg, tk)
    eps2 = (eps.detach() * 1.3).requires_grad_()
    chg2 = (chg.detach() * 0.7).requires_grad_()
    x2 = torch.tensor(X * 1.001, device="cuda", requires_grad=True)
    U2 = model(x2, eps2, sig, chg2, tk)
    U1.sum().backward()
    ref = _oracle_weighted(spec, X.astype(np.float64), np.ones(4))
    for key, t in (("epsilon", eps), ("sigma", sig), ("charge", chg), ("torsion_k", tk)):
        assert _rel(t.grad.cpu().numpy(), ref[key]) < 1e-4, key
    o = oracle.System(dict(spec, n_replicas=2))
    for r in range(4):
        assert _rel(x1.grad[r].cpu().numpy(), -o.eval(X[r])[1]) < 1e-5
    # and the second pass, run backward afterwards, still gets p2's gradient
    U2.sum().backward()
    spec2 = dict(spec, epsilon=np.asarray(spec["epsilon"]) * 1.3, charge=np.asarray(spec["charge"]) * 0.7)
    ref2 = _oracle_weighted(spec2, (X * 1.001).astype(np.float32).astype(np.float64), np.ones(4))
    assert _rel(eps2.grad.cpu().numpy(), ref2["epsilon"]) < 1e-4
    assert _rel(chg2.grad.cpu().numpy(), ref2["charge"]) < 1e-4
