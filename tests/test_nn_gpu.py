"""GPU parity of the surrogate library (libko_nn.so) against the float64 oracle.

Tolerances.  Both sides round the same values to BF16 at the same points; the
device accumulates in float32 (MFMA), the oracle in float64.  A float32 sum of
at most 256 products of magnitude <= 1 differs from float64 by < 256 * 2^-24 of
its magnitude, so a rounded activation differs only where that error straddles
a BF16 rounding boundary, by one BF16 ulp (2^-8 relative) of that element.  Its
effect on y is bounded by 2^-8 * |a| * |w4| per flipped element; with weights of
scale 0.08 and a handful of flips that stays far below 1e-3 (1 + |y|), the
bound used for y.  Gradients pass through the same flips (dZ1..dZ3 are also
rounded), so on random data they are compared per tensor in relative L2 norm
(<= 1e-2).  On a case built so that no rounding happens at all (dyadic
weights and inputs with few significant bits), outputs, loss and every
gradient element must equal the oracle exactly, and one Adam step must land
within one float32 ulp of it, element by element.
"""

import sys

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
nn = pytest.importorskip("paper_1511_07983_amd.nn")


def say(*a):
    print("[nn-gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def make_case(seed, B, n, scale=0.08):
    rng = np.random.default_rng(seed)
    params = {name: rng.normal(0.0, scale, size=shape) for name, shape in mlp.SHAPES}
    flat = mlp.flatten(params).astype(np.float32)
    feat = rng.normal(0.0, 1.0, size=(1, n, mlp.N_FEAT)).astype(np.float32)
    pos = np.stack([rng.permutation(n) for _ in range(B)]).astype(np.uint8)
    if n < 16 and B > 2:
        pos[1, : n // 2] = mlp.UNPLACED  # a partial order: some kernels unplaced
    X = np.zeros((B, n, mlp.D_IN))
    X[:, :, :mlp.N_FEAT] = feat[0][None].astype(np.float64)
    for b in range(B):
        X[b, np.arange(n), mlp.N_FEAT + pos[b]] = 1.0
    return rng, flat, feat, pos, X


def device_tokens(model, feat, pos):
    f = torch.from_numpy(feat).to("cuda:0")
    p = torch.from_numpy(pos).to("cuda:0")
    return model.tokens(f, p)


def bf16_values(x_int16):
    u = x_int16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


@pytest.mark.parametrize("B,n", [(1, 1), (37, 5), (64, 16), (300, 12), (129, 9)])
def test_tokens_and_forward(B, n):
    rng, flat, feat, pos, X = make_case(10 + B + n, B, n)
    say(f"forward B={B} n={n}")
    model = nn.Surrogate(flat)
    x = device_tokens(model, feat, pos)
    assert np.array_equal(bf16_values(x), mlp.bf16(X))
    y = model.forward(x).cpu().numpy().astype(np.float64)
    p64 = mlp.unflatten(flat.astype(np.float64))
    yo, _ = mlp.forward(p64, X)
    err = np.abs(y - yo)
    assert err.max() <= 1e-3 * (1.0 + np.abs(yo).max()), (err.max(), np.abs(yo).max())


@pytest.mark.parametrize("B,n", [(37, 5), (256, 12), (70, 16)])
def test_gradients(B, n):
    rng, flat, feat, pos, X = make_case(20 + B + n, B, n)
    say(f"backward B={B} n={n}")
    model = nn.Surrogate(flat)
    x = device_tokens(model, feat, pos)
    p64 = mlp.unflatten(flat.astype(np.float64))
    yo, _ = mlp.forward(p64, X)
    t = (yo + rng.normal(0.0, 0.5, size=B)).astype(np.float32)
    loss = model.backward(x, torch.from_numpy(t).to("cuda:0"))
    lo, _, go = mlp.loss_and_grads(p64, X, t.astype(np.float64))
    assert float(loss.cpu()[0]) == pytest.approx(lo, rel=1e-3)
    g = mlp.unflatten(model.read("grads").astype(np.float64))
    for name, _ in mlp.SHAPES:
        a, b = g[name].ravel(), go[name].ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 1e-2, (name, rel)


def make_dyadic_case(seed, B, n):
    """A case on which the device's float32 arithmetic is exact: features are
    0 or 1, weights are sparse multiples of 1/4, 1/2 (at most 3, 2 and 1
    nonzeros per row of W1, W2, W3), biases small multiples of a power of two.
    Then every value at a BF16 rounding point (S, A2, A3, dZ1..dZ3) has at most
    8 significant bits and every float32 sum stays below 2^24 units of its
    grid, so the device's outputs and gradients must equal the oracle's float64
    values exactly, whatever the summation order.  B is a power of two and the
    targets differ from the exact outputs by +-1/4 or +-1/2, so dy is exact."""
    rng = np.random.default_rng(seed)
    used = mlp.N_FEAT + mlp.N_POS
    W1 = np.zeros((mlp.D_HID, mlp.D_IN))
    for r in range(mlp.D_HID):
        cols = rng.choice(used, size=3, replace=False)
        W1[r, cols] = rng.choice([-0.25, 0.25], size=3)
    W2 = np.zeros((mlp.D_HID, mlp.D_HID))
    W3 = np.zeros((mlp.D_HID, mlp.D_HID))
    for r in range(mlp.D_HID):
        cols = rng.choice(mlp.D_HID, size=2, replace=False)
        W2[r, cols] = rng.choice([-0.5, 0.5], size=2)
        W3[r, rng.integers(0, mlp.D_HID)] = rng.choice([-0.5, 0.5])
    params = {"W1": W1, "b1": rng.choice([-0.25, 0.0, 0.25], size=mlp.D_HID),
              "W2": W2, "b2": rng.choice([-0.125, 0.0, 0.125], size=mlp.D_HID),
              "W3": W3, "b3": rng.choice([-0.0625, 0.0, 0.0625], size=mlp.D_HID),
              "w4": rng.choice([-0.5, 0.0, 0.5], size=mlp.D_HID), "b4": np.array([0.03125])}
    flat = mlp.flatten(params).astype(np.float32)
    assert np.array_equal(flat.astype(np.float64), mlp.flatten(params))
    feat = rng.integers(0, 2, size=(1, n, mlp.N_FEAT)).astype(np.float32)
    pos = np.stack([rng.permutation(n) for _ in range(B)]).astype(np.uint8)
    pos[1, : n // 2] = mlp.UNPLACED  # a partial order
    X = np.zeros((B, n, mlp.D_IN))
    X[:, :, :mlp.N_FEAT] = feat[0][None].astype(np.float64)
    for b in range(B):
        X[b, np.arange(n), mlp.N_FEAT + pos[b]] = 1.0
    y, c = mlp.forward(params, X)
    # the rounding points really are exact on this case (so the comparison is exact)
    for key in ("Sb", "A2b", "A3b"):
        assert np.array_equal(mlp.bf16(c[key]), c[key]), key
    t = (y + rng.choice([-0.5, -0.25, 0.25, 0.5], size=B)).astype(np.float32)
    assert np.array_equal(t.astype(np.float64) - y, t - y)
    return params, flat, feat, pos, X, y, t


@pytest.mark.parametrize("B,n", [(64, 10), (128, 16), (32, 3)])
def test_gradients_exact_element_by_element(B, n):
    params, flat, feat, pos, X, y_or, t = make_dyadic_case(60 + n, B, n)
    say(f"exact backward B={B} n={n}")
    model = nn.Surrogate(flat)
    x = device_tokens(model, feat, pos)
    assert np.array_equal(bf16_values(x), X)
    y = model.forward(x).cpu().numpy().astype(np.float64)
    assert np.array_equal(y, y_or)
    loss = model.backward(x, torch.from_numpy(t).to("cuda:0"))
    lo, _, go = mlp.loss_and_grads(params, X, t.astype(np.float64))
    # the oracle's own rounding points are identities here as well
    _, _, go_plain = mlp.loss_and_grads(params, X, t.astype(np.float64), bf16_points=False)
    assert float(loss.cpu()[0]) == lo
    g = mlp.unflatten(model.read("grads").astype(np.float64))
    for name, _ in mlp.SHAPES:
        assert np.array_equal(go[name], go_plain[name]), name
        bad = np.flatnonzero(g[name].ravel() != go[name].ravel())
        assert bad.size == 0, (name, bad[:5], g[name].ravel()[bad[:5]], go[name].ravel()[bad[:5]])
    assert sum(np.count_nonzero(go[k]) for k, _ in mlp.SHAPES) > 2000  # the case is not trivial
    # one Adam step from the same float32 weights and exact gradients, element
    # by element: the device evaluates the update (moments, bias corrections,
    # square root, epsilon, quotient, learning rate: about ten float32
    # roundings of relative size 2^-24 each) and rounds the new weight, so it
    # lies within one float32 ulp of the new weight plus 10 * 2^-24 * lr of
    # the oracle's float64 step; components with a zero gradient do not move
    lr = 1e-3
    model.adam(1, lr)
    w_dev = model.read("weights").astype(np.float64)
    gflat = mlp.flatten(go)
    w0 = flat.astype(np.float64)
    w_or, _, _ = mlp.adam_step(w0, gflat, np.zeros_like(gflat), np.zeros_like(gflat), 1, lr)
    ulp = np.spacing(np.abs(w_or).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(w_dev - w_or) <= ulp + 10 * 2.0 ** -24 * lr), np.abs(w_dev - w_or).max()
    assert np.array_equal(w_dev[gflat == 0], w0[gflat == 0])


def test_adam_step():
    """One Adam step from the loaded weights: well-conditioned components (not
    near a zero gradient, where the first step is lr * sign(g)) match the oracle;
    every component moves by at most lr."""
    B, n, lr = 96, 8, 1e-3
    rng, flat, feat, pos, X = make_case(31, B, n)
    model = nn.Surrogate(flat)
    x = device_tokens(model, feat, pos)
    p64 = mlp.unflatten(flat.astype(np.float64))
    yo, _ = mlp.forward(p64, X)
    t = (yo + rng.normal(0.0, 0.5, size=B)).astype(np.float32)
    model.backward(x, torch.from_numpy(t).to("cuda:0"))
    model.adam(1, lr)
    w_dev = model.read("weights").astype(np.float64)
    _, _, go = mlp.loss_and_grads(p64, X, t.astype(np.float64))
    g = mlp.flatten(go)
    w0 = flat.astype(np.float64)
    w_or, _, _ = mlp.adam_step(w0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    assert np.abs(w_dev - w0).max() <= lr * (1 + 1e-5)
    good = np.abs(g) > 1e-2 * np.abs(g).max()
    assert good.sum() > 1000
    assert np.allclose(w_dev[good], w_or[good], rtol=0, atol=1e-6)


def test_training_reduces_loss():
    """Fit targets produced by a random teacher network: 300 Adam steps cut the
    loss by at least 10x."""
    B, n = 512, 10
    rng = np.random.default_rng(41)
    teacher = {name: rng.normal(0.0, 0.1, size=shape) for name, shape in mlp.SHAPES}
    _, flat, feat, _, _ = make_case(42, 2, n)
    pos = np.stack([rng.permutation(n) for _ in range(B)]).astype(np.uint8)
    X = np.zeros((B, n, mlp.D_IN))
    X[:, :, :mlp.N_FEAT] = feat[0][None].astype(np.float64)
    for b in range(B):
        X[b, np.arange(n), mlp.N_FEAT + pos[b]] = 1.0
    t, _ = mlp.forward(teacher, X, bf16_points=False)
    t = ((t - t.mean()) / (t.std() + 1e-12)).astype(np.float32)
    model = nn.Surrogate(flat)
    x = device_tokens(model, feat, pos)
    td = torch.from_numpy(t).to("cuda:0")
    first = float(model.backward(x, td).cpu()[0])
    model.adam(1, 3e-3)
    for step in range(2, 301):
        loss = model.backward(x, td)
        model.adam(step, 3e-3)
    last = float(loss.cpu()[0])
    say(f"training loss {first:.4f} -> {last:.4f}")
    assert last < first / 10


@pytest.mark.parametrize("B,n", [(1, 1), (77, 6), (513, 12), (64, 16), (300, 9)])
def test_forward_positions_matches_oracle_and_token_path(B, n):
    """Scoring path: the layer-1 table equals the oracle's per-token first
    layer, and y from positions matches the oracle and the token path."""
    rng, flat, feat, pos, X = make_case(50 + B + n, B, n)
    say(f"forward from positions B={B} n={n}")
    model = nn.Surrogate(flat)
    table = model.layer1_table(torch.from_numpy(feat[0]).to("cuda:0")).cpu().numpy().astype(np.float64)
    p64 = mlp.unflatten(flat.astype(np.float64))
    Xtab = np.zeros((n, mlp.N_POS, mlp.D_IN))
    Xtab[:, :, :mlp.N_FEAT] = feat[0][:, None, :].astype(np.float64)
    for q in range(mlp.N_POS):
        Xtab[:, q, mlp.N_FEAT + q] = 1.0
    want = np.maximum(mlp.bf16(Xtab) @ mlp.bf16(p64["W1"]).T + p64["b1"], 0.0)
    assert np.abs(table - want).max() <= 1e-5 * (1.0 + np.abs(want).max())
    y = model.forward_positions(torch.from_numpy(table.astype(np.float32)).to("cuda:0"),
                                torch.from_numpy(pos).to("cuda:0")).cpu().numpy().astype(np.float64)
    yo, _ = mlp.forward(p64, X)
    assert np.abs(y - yo).max() <= 1e-3 * (1.0 + np.abs(yo).max())
    y_tok = model.forward(device_tokens(model, feat, pos)).cpu().numpy().astype(np.float64)
    assert np.abs(y - y_tok).max() <= 1e-3 * (1.0 + np.abs(y_tok).max())


@pytest.mark.parametrize("B,n", [(1, 1), (63, 5), (64, 16), (65, 12), (1000, 12), (4097, 9), (300, 16)])
def test_fused_score_equals_table_path_bit_for_bit(B, n):
    """ko_nn_score (one kernel: layer-1 pooling from features and position
    weights, both MFMA layers, output layer) against the table path (layer-1
    table, gather-sum, two GEMM launches, output kernel): every y identical,
    on ragged tiles, partial orders and out-of-range positions; and within
    the oracle's tolerance."""
    rng, flat, feat, pos, X = make_case(70 + B + n, B, n)
    if B > 3:
        pos[2, :] = 200  # positions above 16 count as unplaced
        X[2, :, mlp.N_FEAT:] = 0.0
        X[2, :, mlp.N_FEAT + mlp.UNPLACED] = 1.0
    say(f"fused score B={B} n={n}")
    model = nn.Surrogate(flat)
    f = torch.from_numpy(feat[0]).to("cuda:0")
    p = torch.from_numpy(pos).to("cuda:0")
    y_fused = model.score(f, p).cpu().numpy()
    y_table = model.forward_positions(model.layer1_table(f), p).cpu().numpy()
    bad = np.flatnonzero(y_fused.view(np.uint32) != y_table.view(np.uint32))
    assert bad.size == 0, (bad[:5], y_fused[bad[:5]], y_table[bad[:5]])
    # against the oracle with the tolerance of the module docstring, which
    # allows a handful of BF16 rounding flips per row: it holds for a few
    # hundred rows; over thousands, some row collects more flips (the table
    # path, identical above, does the same)
    m = min(B, 256)
    yo, _ = mlp.forward(mlp.unflatten(flat.astype(np.float64)), X[:m])
    assert np.abs(y_fused[:m] - yo).max() <= 1e-3 * (1.0 + np.abs(yo).max())


def _split_bf16(T):
    """hi = bf16(T), lo = bf16(T - hi) of float32 values, both as float64."""
    T = np.asarray(T, dtype=np.float32)
    hi = mlp.bf16(T)
    lo = mlp.bf16((T.astype(np.float64) - hi).astype(np.float32))
    return hi, lo


def _unfrag(raw, ks):
    """A [256, 32 ks] BF16 matrix (uint16) from its MFMA fragment order:
    element (h, k) at ((h // 16) ks + k // 32) 512 + (16 ((k % 32) // 8) +
    h % 16) 8 + k % 8."""
    return raw.reshape(16, ks, 4, 16, 8).transpose(0, 3, 1, 2, 4).reshape(16 * 16, ks * 32)


def _bf16_bits_to_f64(u16):
    return (u16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _slot_table(T, n):
    """Rows of the layer-1 table T [n, 17, 256] in slot order: kernel i's
    slots are its positions 0..n-1, then "unplaced" (16)."""
    slots = list(range(n)) + [mlp.UNPLACED]
    return T[:, slots, :].reshape(n * (n + 1), mlp.D_HID)


@pytest.mark.parametrize("B,n", [(1, 1), (63, 5), (64, 16), (65, 12), (1000, 12), (4097, 9), (300, 16)])
def test_split_score_matches_its_definition_and_oracle(B, n):
    """ko_nn_score_split (pooling as a one-hot MFMA product with the table in
    BF16 high and low parts, n + 1 slots per kernel): the operand pack holds
    exactly hi = bf16(T) and lo = bf16(T - hi) of the layer-1 table in slot
    order and the BF16 W2 and W3, each in fragment order.  y is compared with the oracle's layers applied to S = sum over
    kernels of (hi + lo) (float64 sums), the path's definition: the device's S
    differs from it only by float32 accumulation, so a row differs only where
    that moves S across a BF16 rounding boundary (as for every path): at most
    1% of the rows (or 2) by more than 1e-5 (1 + |y|), none by more than 1e-2
    (1 + |y|).  Against the token model the 2^-17 representation of T adds about
    one such BF16 flip of S per row (probability about 2^-8 per element),
    each moving y by at most 2^-8 of one S element's contribution: every row
    of the first 256 within 1e-2 (1 + max |y|)."""
    rng, flat, feat, pos, X = make_case(90 + B + n, B, n)
    if B > 3:
        pos[2, :] = 200  # positions above 16 count as unplaced
        X[2, :, mlp.N_FEAT:] = 0.0
        X[2, :, mlp.N_FEAT + mlp.UNPLACED] = 1.0
    say(f"split score B={B} n={n}")
    model = nn.Surrogate(flat)
    f = torch.from_numpy(feat[0]).to("cuda:0")
    p = torch.from_numpy(pos).to("cuda:0")
    T = model.layer1_table(f).cpu().numpy()                     # [n, 17, 256] float32
    split = model.split_table(f)
    K1 = n * (n + 1)
    KP = -(-K1 // 32) * 32
    raw = split.cpu().numpy().view(np.uint16)
    assert raw.size == 2 * 256 * KP + 2 * 256 * 256
    got = np.stack([_bf16_bits_to_f64(_unfrag(raw[q * 256 * KP:(q + 1) * 256 * KP], KP // 32)) for q in (0, 1)])
    Ts = _slot_table(T, n)                                      # [K1, 256]
    hi, lo = _split_bf16(Ts.T)                                  # [256, K1]
    assert np.array_equal(got[0, :, :K1], hi) and np.array_equal(got[1, :, :K1], lo)
    assert not got[:, :, K1:].any()
    # the pack's copies of W2 and W3: the BF16 weights, in fragment order
    pw = mlp.unflatten(flat.astype(np.float64))
    off = 2 * 256 * KP
    for q, name in enumerate(("W2", "W3")):
        w = _bf16_bits_to_f64(_unfrag(raw[off + q * 65536:off + (q + 1) * 65536], 8))
        assert np.array_equal(w, mlp.bf16(pw[name])), name
    assert np.abs(hi + lo - Ts.T).max() <= 2.0 ** -17 * np.abs(Ts).max()
    y = model.score_split(split, p).cpu().numpy().astype(np.float64)
    slot = np.where(pos.astype(np.int64) < n, pos.astype(np.int64), n)
    S = (hi + lo).T[np.arange(n)[None, :] * (n + 1) + slot].sum(axis=1)  # [B, 256]
    p64 = mlp.unflatten(flat.astype(np.float64))
    ys, _ = mlp.from_pooled(p64, S)
    err = np.abs(y - ys)
    flips = int(np.sum(err > 1e-5 * (1.0 + np.abs(ys))))
    assert flips <= max(2, 0.01 * B), (flips, err.max())
    assert np.all(err <= 1e-2 * (1.0 + np.abs(ys))), err.max()
    m = min(B, 256)
    yo, _ = mlp.forward(p64, X[:m])
    assert np.abs(y[:m] - yo).max() <= 1e-2 * (1.0 + np.abs(yo).max())


def test_split_pack_follows_the_weights():
    """The operand pack holds a copy of W2 and W3: a pack made after an Adam
    step carries the updated BF16 weights (and scores with them), the pack made
    before keeps the old ones."""
    B, n = 300, 9
    rng, flat, feat, pos, X = make_case(17, B, n)
    model = nn.Surrogate(flat)
    f = torch.from_numpy(feat[0]).to("cuda:0")
    p = torch.from_numpy(pos).to("cuda:0")
    before = model.split_table(f).cpu().numpy().view(np.uint16)
    x = device_tokens(model, feat, pos)
    t = torch.from_numpy(rng.normal(0.0, 1.0, size=B).astype(np.float32)).to("cuda:0")
    model.backward(x, t)
    model.adam(1, 1e-2)
    after_t = model.split_table(f)
    after = after_t.cpu().numpy().view(np.uint16)
    KP = -(-n * (n + 1) // 32) * 32
    off = 2 * 256 * KP
    pw = mlp.unflatten(model.read("weights").astype(np.float64))
    for q, name in enumerate(("W2", "W3")):
        blk = slice(off + q * 65536, off + (q + 1) * 65536)
        assert np.array_equal(_bf16_bits_to_f64(_unfrag(after[blk], 8)), mlp.bf16(pw[name])), name
        assert not np.array_equal(after[blk], before[blk]), name
    # scores from the new pack are the new model's (within the split path's tolerance)
    y = model.score_split(after_t, p).cpu().numpy().astype(np.float64)
    yo, _ = mlp.forward(pw, X[:256])
    assert np.abs(y[:256] - yo).max() <= 1e-2 * (1.0 + np.abs(yo).max())


def test_split_score_flags_positions_outside_the_set():
    """A position in n..15 is no launch position of an n-kernel order: that
    row's y is NaN and the other rows are as without it.  The tile's thread t
    reads position bytes t, t + 256, ... (row-major, n per row) and thread r
    clears row r's flag: rows 11 and 21 of the first tile have their bad
    position read by a thread of another wave than the one that clears the
    flag (bytes 68 and 130 at n = 6)."""
    B, n = 200, 6
    rng, flat, feat, pos, X = make_case(7, B, n)
    model = nn.Surrogate(flat)
    f = torch.from_numpy(feat[0]).to("cuda:0")
    split = model.split_table(f)
    y0 = model.score_split(split, torch.from_numpy(pos).to("cuda:0")).cpu().numpy()
    bad = pos.copy()
    bad[3, 2] = 9
    bad[11, 2] = 7
    bad[21, 4] = 12
    bad[150, 0] = 15
    rows = [3, 11, 21, 150]
    y1 = model.score_split(split, torch.from_numpy(bad).to("cuda:0")).cpu().numpy()
    assert np.all(np.isnan(y1[rows])), y1[rows]
    keep = np.setdiff1d(np.arange(B), rows)
    assert np.isfinite(y0).all() and np.array_equal(y0[keep], y1[keep])


def test_split_score_accumulates_an_ensemble_mean():
    """ko_nn_score_split_acc: the first member writes scale * score, the others
    add scale * score in order; against the members' own scores combined the
    same way in float32 (the device may fuse each multiply-add: one rounding
    instead of two, within 2 ulp of the result)."""
    B, n = 700, 12
    models, splits, own = [], [], []
    rng, _, feat, pos, _ = make_case(5, B, n)
    f = torch.from_numpy(feat[0]).to("cuda:0")
    p = torch.from_numpy(pos).to("cuda:0")
    for k in range(3):
        _, flat, _, _, _ = make_case(30 + k, 1, n)
        m = nn.Surrogate(flat)
        models.append(m)
        splits.append(m.split_table(f))
        own.append(m.score_split(splits[-1], p).cpu().numpy())
    scale = np.float32(1.0 / 3.0)
    y = None
    for k, (m, t) in enumerate(zip(models, splits)):
        y = m.score_split(t, p, y=y, scale=float(scale), accumulate=k > 0)
    y = y.cpu().numpy()
    want = scale * own[0]
    for k in (1, 2):
        want = want + scale * own[k]
    assert np.all(np.abs(y - want) <= 2 * np.spacing(np.abs(want).astype(np.float32))), np.abs(y - want).max()
    assert not np.array_equal(own[0], own[1])
