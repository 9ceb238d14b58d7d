"""GPU checks of the learned auxiliary: the MLP's hand-written forward, backward and
Adam kernels against the oracle's NumPy network (FP32 kernels vs FP64 reference
on the same FP32 parameters and data), rz_set_aux against the oracle relaxation
with the same weights, and what a trained network gains over the cell-averaged
weights on a held-out mesh."""
import numpy as np
import pytest

import synth
from oracle.lattice import Mesh, Lattice
from oracle import auxop, schwarz, learned

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14284_amd import rz as mod
    return mod


@pytest.fixture(scope="module")
def ctx(rz):
    return rz.Context(0, torch.cuda.current_stream())


def pack(P):
    return np.concatenate([q.ravel() for q in P]).astype(np.float32)


def unpack(v, nin, nh, no):
    shapes = [(nh, nin), (nh,), (nh, nh), (nh,), (no, nh), (no,)]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(v[o:o + n].reshape(s).astype(np.float64))
        o += n
    return out


def data(n, seed):
    X = (0.3 * synth.uniform_pm1(seed, n * 51)).reshape(n, 51).astype(np.float32)
    Y = (0.1 * synth.uniform_pm1(seed + 1, n * 6)).reshape(n, 6).astype(np.float32)
    return X, Y


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def test_mlp_init_matches_oracle(rz, ctx):
    m = rz.MLP(ctx, 51, 64, 6, seed=5)
    assert np.allclose(m.params(), pack(learned.init_params(51, 64, 6, 5)), rtol=1e-6, atol=1e-7)


def test_mlp_forward_backward_adam_parity(rz, ctx):
    m = rz.MLP(ctx, 51, 32, 6, seed=9)
    P = unpack(m.params(), 51, 32, 6)
    X, Y = data(300, 21)
    Xd, Yd = dev(X), dev(Y)
    # forward
    out = torch.empty((300, 6), dtype=torch.float32, device="cuda:0")
    m.predict(Xd, out)
    y_ref, _ = learned.forward(P, X.astype(np.float64))
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy() - y_ref).max() < 1e-5 * max(1.0, np.abs(y_ref).max())
    # loss and gradient
    loss, g = m.loss_grad(Xd, Yd)
    loss_ref, g_ref = learned.loss_and_grads(P, X.astype(np.float64), Y.astype(np.float64))
    assert abs(loss - loss_ref) < 1e-5 * loss_ref
    gr = pack(g_ref).astype(np.float64)
    assert np.linalg.norm(g - gr) < 1e-4 * np.linalg.norm(gr)
    # one Adam step (first step)
    m.adam_step(Xd, Yd, 1e-3)
    mm = [np.zeros_like(q) for q in P]
    vv = [np.zeros_like(q) for q in P]
    P2 = learned.adam_step([q.copy() for q in P], g_ref, mm, vv, 1, 1e-3)
    assert np.abs(m.params() - pack(P2)).max() < 2e-5


def test_set_aux_relax_parity(rz, ctx):
    n, p = 3, 4
    v = synth.perturbed_vertices(n, 3)
    a = synth.c5_coefficient_samples(v, n)
    b = np.ones_like(a)
    pb = rz.Problem(ctx, n, p, a, b, vertices=v, omega=0.3)
    t, _, base = pb.aux_data()
    pb.set_aux(t)
    assert np.array_equal(pb.aux_coefficients(), t)
    m = Mesh(n, n, n, vertices=v)
    lat = Lattice(m, "grad", p)
    R = schwarz.SCRelaxGrad(lat, auxop.separable_operator(lat, t))
    r = np.where(lat.dirichlet_mask(), 0.0, synth.uniform_pm1(13, lat.ndofs))
    z = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
    pb.relax(dev(r), z)
    torch.cuda.synchronize()
    z_ref = R.apply(r)
    zc = z.cpu().numpy()
    assert np.linalg.norm(zc - z_ref) < 1e-12 * np.linalg.norm(z_ref)
    assert np.abs(zc - z_ref).max() < 1e-12 * np.abs(z_ref).max()


def _cells(rz, n, p, seed):
    v = synth.perturbed_vertices(n, seed)
    a = synth.c5_coefficient_samples(v, n)
    pb = rz.Problem(rz.Context(-1), n, p, a, 1.0, vertices=v)
    t, f, base = pb.aux_data()
    return f.astype(np.float32), np.log(t / base).astype(np.float32), t, base


def test_trained_network_beats_cell_average_on_held_out_mesh(rz, ctx):
    # train on meshes with seeds 10..13, evaluate on the seed-3 mesh
    n, p = 8, 6
    parts = [_cells(rz, n, p, s) for s in range(10, 14)]
    X = np.concatenate([q[0] for q in parts])
    Y = np.concatenate([q[1] for q in parts])
    m = rz.MLP(ctx, 51, 64, 6, seed=1)
    loss0, _ = m.loss_grad(dev(X), dev(Y))
    loss = m.train(dev(X), dev(Y), epochs=60, batch=256, lr=2e-3, seed=11)
    assert loss < 0.2 * loss0
    Xt, Yt, t, base = _cells(rz, n, p, 3)
    out = torch.empty((Xt.shape[0], 6), dtype=torch.float32, device="cuda:0")
    m.predict(dev(Xt), out)
    torch.cuda.synchronize()
    pred = out.cpu().numpy().astype(np.float64)
    err_mlp = np.sqrt(np.mean((pred - Yt) ** 2))
    err_avg = np.sqrt(np.mean(Yt.astype(np.float64) ** 2))   # the cell average predicts log-ratio 0
    assert err_mlp < 0.5 * err_avg, (err_mlp, err_avg)
