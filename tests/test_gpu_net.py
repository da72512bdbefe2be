"""GPU parity of the candidate classifier: stamp extraction (bit-exact FP16), forward logits,
loss and every parameter's gradient against the FP64 oracle (oracle/net.py), and Adam steps.

The oracle gets the same FP16 stamps and the FP16-rounded convolution weights the kernels
multiply with (biases and the linear unit stay FP32 on both sides), so the remaining
differences are the kernels' FP16 storage of the first two layers' activations and of the
back-propagated gradients (relative rounding <= 2^-11 each, a few roundings deep) and FP32
accumulation.  Bars (derived from that, with margin for cancellation in the sums):
  logits      |dz| <= 4e-3 max|z| + 1e-4
  loss        relative 1e-3
  gradients   per tensor: max-abs <= 1e-2 of the tensor's largest |g|, L2 <= 1e-2 relative
              (measured worst over the cases: 6.0e-3 and 5.1e-3)
  Adam        relative 1e-5 (FP32 against FP64 arithmetic on the same inputs)
"""
import numpy as np
import pytest

import synth
from oracle import net as onet

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2606_04304_amd as nb  # noqa: E402

DEV = torch.device("cuda", 0)


def _rounded_theta(theta32):
    """The parameters as the kernels use them: convolution weights rounded to FP16."""
    p = onet.unpack(theta32.astype(np.float64))
    for k in ("W1", "W2", "W3"):
        p[k] = p[k].astype(np.float16).astype(np.float64)
    return onet.pack(p)


def _stamps(n, seed, scale=1.0, sparse=False):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 33, 9, 9)) * scale
    if sparse:  # spiky stamps like the detector's: mostly noise, a bright core
        x[:, 16, 3:6, 3:6] += rng.uniform(5, 20, size=(n, 1, 1))
    return x.astype(np.float16)


def test_stamps_bit_exact():
    print("net stamps", flush=True)
    rng = np.random.default_rng(11)
    C, N = 70, 40
    cube = (rng.standard_normal((C, N, N)) * 30).astype(np.float32)
    cube[5, 7, 9] = 1e6  # saturates at the FP16 maximum
    cands = [(0, 0, 0), (69, 39, 39), (35, 20, 17), (5, 7, 9), (16, 4, 4), (53, 35, 2)]
    rec = np.zeros((len(cands), 5), dtype=np.int32)
    for k, (c, y, x) in enumerate(cands):
        rec[k, :4] = (x, y, c, 1)
    got = nb.nbsi_stamps(torch.from_numpy(cube).to(DEV), torch.from_numpy(rec).to(DEV)).cpu().numpy()
    ref = onet.stamps(cube.astype(np.float64), cands)
    ref = np.clip(ref, -65504, 65504).astype(np.float16)
    assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))
    assert nb.nbsi_stamps(torch.from_numpy(cube).to(DEV), torch.zeros((0, 5), dtype=torch.int32, device=DEV)).shape[0] == 0


@pytest.mark.parametrize("n,seed", [(1, 1), (7, 2), (64, 3), (300, 4)])
def test_forward_matches_oracle(n, seed):
    print(f"net forward n={n}", flush=True)
    theta = synth.net_init(100 + seed)
    theta[onet.N_PARAM - 1 - 32 - 32:onet.N_PARAM - 1 - 32] = 0.05  # small positive b3
    x = _stamps(n, seed, sparse=(seed % 2 == 0))
    net = nb.Net(theta, max_batch=512)
    z = net.forward(torch.from_numpy(x).to(DEV)).cpu().numpy()
    zr, _ = onet.forward(_rounded_theta(theta), x.astype(np.float64))
    assert np.abs(z - zr).max() <= 4e-3 * np.abs(zr).max() + 1e-4, (z[:4], zr[:4])
    net.close()


def test_forward_with_index_and_empty_entries():
    print("net forward index", flush=True)
    theta = synth.net_init(7)
    x = _stamps(10, 5)
    net = nb.Net(theta, max_batch=64)
    idx = torch.tensor([9, 0, 3, 3, -1, 10], dtype=torch.int32, device=DEV)
    z = net.forward(torch.from_numpy(x).to(DEV), index=idx).cpu().numpy()
    xs = np.stack([x[9], x[0], x[3], x[3], np.zeros_like(x[0]), np.zeros_like(x[0])])
    zr, _ = onet.forward(_rounded_theta(theta), xs.astype(np.float64))
    assert np.abs(z - zr).max() <= 4e-3 * np.abs(zr).max() + 1e-4
    assert z[2] == z[3] and z[4] == z[5]
    net.close()


def _check_grads(g, gr):
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in onet.SHAPES])
    for k, (name, _) in enumerate(onet.SHAPES):
        a, b = g[offs[k]:offs[k + 1]], gr[offs[k]:offs[k + 1]]
        peak = np.abs(b).max()
        if peak == 0:
            assert np.abs(a).max() == 0, name
            continue
        print(f"  {name}: max-abs {np.abs(a - b).max() / peak:.2e} of peak, "
              f"L2 {np.linalg.norm(a - b) / np.linalg.norm(b):.2e}", flush=True)
        assert np.abs(a - b).max() <= 1e-2 * peak, (name, np.abs(a - b).max() / peak)
        assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b), (name, np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,seed", [(3, 21), (50, 22), (257, 23)])
def test_gradient_matches_oracle(n, seed):
    print(f"net grad n={n}", flush=True)
    theta = synth.net_init(200 + seed)
    p = onet.unpack(theta.astype(np.float64))
    rng = np.random.default_rng(seed)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.uniform(-0.05, 0.1, size=p[k].shape)
    theta = onet.pack(p).astype(np.float32)
    x = _stamps(n, seed, sparse=True)
    y = (rng.random(n) < 0.4).astype(np.float32)
    net = nb.Net(theta, max_batch=512)
    loss, g = net.grad(torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV))
    loss, g = float(loss.item()), g.cpu().numpy().astype(np.float64)
    lr_, gr = onet.loss_and_grad(_rounded_theta(theta), x.astype(np.float64), y.astype(np.float64))
    assert abs(loss - lr_) <= 1e-3 * abs(lr_), (loss, lr_)
    _check_grads(g, gr)
    net.close()


def test_gradient_with_index_and_labels_indexed():
    print("net grad index", flush=True)
    theta = synth.net_init(31)
    x = _stamps(40, 31, sparse=True)
    rng = np.random.default_rng(31)
    y = (rng.random(40) < 0.5).astype(np.float32)
    idx = rng.integers(0, 40, size=25).astype(np.int32)
    net = nb.Net(theta, max_batch=64)
    loss, g = net.grad(torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV),
                       index=torch.from_numpy(idx).to(DEV))
    lr_, gr = onet.loss_and_grad(_rounded_theta(theta), x[idx].astype(np.float64), y[idx].astype(np.float64))
    assert abs(loss.item() - lr_) <= 1e-3 * abs(lr_)
    _check_grads(g.cpu().numpy().astype(np.float64), gr)
    net.close()


def test_adam_matches_oracle():
    print("net adam", flush=True)
    theta = synth.net_init(41)
    rng = np.random.default_rng(41)
    net = nb.Net(theta, max_batch=8)
    t64, m, v = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    for step in range(1, 4):
        g = (rng.standard_normal(theta.size) * 10.0 ** rng.uniform(-4, 0, size=theta.size)).astype(np.float32)
        net.adam(torch.from_numpy(g).to(DEV), lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8)
        t64, m, v = onet.adam(t64, m, v, g.astype(np.float64), step, lr=1e-3)
    got = net.get_params().astype(np.float64)
    assert np.abs(got - t64).max() <= 1e-5 * max(1.0, np.abs(t64).max())
    # set_params resets the optimizer: the next step is again a sign step
    net.set_params(theta)
    g = np.full(theta.size, 3.0, dtype=np.float32)
    net.adam(torch.from_numpy(g).to(DEV), lr=0.01)
    np.testing.assert_allclose(net.get_params(), theta - 0.01, rtol=0, atol=2e-6)
    net.close()


def test_train_step_lowers_the_loss():
    """A few hundred steps on a fixed, separable toy batch (a bright centre voxel or not)."""
    print("net train toy", flush=True)
    rng = np.random.default_rng(51)
    n = 256
    x = (rng.standard_normal((n, 33, 9, 9)) * 0.5).astype(np.float32)
    y = (rng.random(n) < 0.5).astype(np.float32)
    x[y == 1, 16, 4, 4] += 8.0
    xs = torch.from_numpy(x.astype(np.float16)).to(DEV)
    ys = torch.from_numpy(y).to(DEV)
    net = nb.Net(synth.net_init(52), max_batch=n)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    first = None
    for it in range(150):
        net.train_step(xs, ys, lr=2e-3, loss=loss)
        if it == 0:
            first = loss.item()
    last = loss.item()
    z = net.forward(xs).cpu().numpy()
    acc = np.mean((z > 0) == (y > 0.5))
    assert last < 0.2 * first and acc > 0.97, (first, last, acc)
    net.close()


def test_net_rejects_bad_arguments():
    net = nb.Net(synth.net_init(1), max_batch=4)
    x = torch.zeros((8, 33, 9, 9), dtype=torch.float16, device=DEV)
    with pytest.raises(nb.NbsiError):
        net.forward(x)  # 8 > max_batch
    with pytest.raises(nb.NbsiError):
        net.forward(x[:2], n=3)  # more rows than stamps without an index
    net.close()
