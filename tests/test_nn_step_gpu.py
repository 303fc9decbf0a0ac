"""GPU checks of the on-device training step (ko_nn_train_step, ko_nn_batch,
ko_nn_step_capture).

The step is the same arithmetic as ko_nn_backward followed by ko_nn_adam, so
the comparisons are bit for bit: gradients, weights and both Adam moments
after each step, and the loss.  The schedule's rate is the one place where
the device evaluates a formula the host also knows (a cosine); there the
step's weights are compared with backward + adam at the host's rate to one
float32 ulp of each weight plus 8 * 2^-24 * lr (the two rates differ by a few
ulp and an Adam update is at most about lr in size).  The graph is replayed
several times with host reads and a permutation rewrite between replays, and
every replay is checked against the eager step (the graph holds no memset
node: every buffer is written by a kernel).
"""

import math
import sys

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
nn = pytest.importorskip("paper_1511_07983_amd.nn")


def say(*a):
    print("[nn-step-gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def params(seed, scale=0.08):
    rng = np.random.default_rng(seed)
    p = {name: rng.normal(0.0, scale, size=shape) for name, shape in mlp.SHAPES}
    return mlp.flatten(p).astype(np.float32)


def sample_tables(seed, S, per, n):
    """feat [S, n, 8], positions [S per, n] (some partial), set_of, makespans,
    per-set centre and scale, as device tensors."""
    rng = np.random.default_rng(seed)
    R = S * per
    feat = rng.normal(0.0, 1.0, size=(S, n, mlp.N_FEAT)).astype(np.float32)
    pos = np.stack([rng.permutation(n) for _ in range(R)]).astype(np.uint8)
    part = rng.random(R) < 0.2
    pos[part, : n // 2] = mlp.UNPLACED
    set_of = np.repeat(np.arange(S, dtype=np.int32), per)
    ms = rng.integers(10_000, 20_000, size=R).astype(np.int64)
    center = rng.integers(9_000, 10_000, size=S).astype(np.int64)
    scale = rng.integers(500, 2_000, size=S).astype(np.int64)
    d = lambda a: torch.from_numpy(a).to("cuda:0")
    return d(feat), d(pos), d(set_of), d(ms), d(center), d(scale)


def host_rate(lr, warmup, total, lr_final, s):
    if s <= warmup:
        return lr * s / max(1, warmup)
    p = (s - warmup) / max(1, total - warmup)
    return lr * (lr_final + (1.0 - lr_final) * 0.5 * (1.0 + math.cos(math.pi * p)))


def state_of(model):
    return {k: model.read(k) for k in ("weights", "grads", "m", "v")}


def assert_same(a, b, what):
    for k in a:
        bad = np.flatnonzero(a[k].view(np.uint32) != b[k].view(np.uint32))
        assert bad.size == 0, (what, k, bad[:5], a[k][bad[:5]], b[k][bad[:5]])


@pytest.mark.parametrize("B,n", [(256, 12), (37, 5), (64, 16)])
def test_train_step_equals_backward_then_adam(B, n):
    say(f"train_step vs backward+adam B={B} n={n}")
    flat = params(100 + B)
    feat, pos, set_of, ms, center, scale = sample_tables(200 + B, 1, B, n)
    a = nn.Surrogate(flat)
    b = nn.Surrogate(flat)
    x = a.tokens(feat, pos, set_of)
    t = a.targets(ms, center, scale, set_of)
    lr = 2e-3
    sch = nn.sched(lr=lr, warmup=0, total=100, lr_final=1.0)   # constant rate lr
    for step in range(1, 4):
        la = a.backward(x, t)
        a.adam(step, lr)
        lb = b.train_step(x, t, sch)
        torch.cuda.synchronize()
        assert float(la.cpu()[0]) == float(lb.cpu()[0]), step
        assert_same(state_of(a), state_of(b), f"step {step}")
        assert nn.sched_read(sch)["step"] == step


@pytest.mark.parametrize("s,warmup,total,lr_final", [(1, 3, 50, 0.05), (3, 3, 50, 0.05), (4, 3, 50, 0.05),
                                                     (30, 3, 50, 0.05), (50, 3, 50, 0.05), (7, 0, 10, 0.2)])
def test_schedule_rate(s, warmup, total, lr_final):
    say(f"schedule s={s} warmup={warmup} total={total}")
    B, n = 128, 8
    flat = params(7)
    feat, pos, set_of, ms, center, scale = sample_tables(8, 1, B, n)
    a = nn.Surrogate(flat)
    b = nn.Surrogate(flat)
    x = a.tokens(feat, pos, set_of)
    t = a.targets(ms, center, scale, set_of)
    lr = 1e-3
    rate = float(np.float32(host_rate(lr, warmup, total, lr_final, s)))
    a.backward(x, t)
    a.adam(s, rate)
    sch = nn.sched(lr=lr, warmup=warmup, total=total, lr_final=lr_final, step=s - 1)
    b.train_step(x, t, sch)
    torch.cuda.synchronize()
    assert nn.sched_read(sch)["step"] == s
    wa, wb = a.read("weights").astype(np.float64), b.read("weights").astype(np.float64)
    ulp = np.spacing(np.abs(wa).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(wa - wb) <= ulp + 8 * 2.0 ** -24 * lr), np.abs(wa - wb).max()
    assert np.abs(wa - flat).max() > 0.1 * rate   # the step moved the weights


def test_batch_selects_rows_of_the_permutation():
    S, per, n, B = 3, 40, 9, 16
    feat, pos, set_of, ms, center, scale = sample_tables(9, S, per, n)
    model = nn.Surrogate(params(9))
    rng = np.random.default_rng(3)
    per_epoch = (S * per) // B
    perm = torch.from_numpy(rng.permutation(S * per)[:per_epoch * B].astype(np.int64)).to("cuda:0")
    for step in (0, 1, per_epoch - 1, per_epoch, 2 * per_epoch + 3):
        say(f"batch step={step}")
        sch = nn.sched(lr=1e-3, per_epoch=per_epoch, step=step)
        x, t = model.batch(feat, pos, set_of, ms, center, scale, perm, sch, B)
        j = step % per_epoch
        rows = perm[j * B:(j + 1) * B].contiguous()
        x2 = model.tokens(feat, pos, set_of, rows=rows)
        t2 = model.targets(ms, center, scale, set_of, rows=rows)
        torch.cuda.synchronize()
        assert torch.equal(x, x2) and torch.equal(t, t2), step
        assert nn.sched_read(sch)["step"] == step   # choosing a batch does not advance the step


def test_graph_replays_equal_eager_steps():
    S, per, n, B = 4, 48, 10, 32
    feat, pos, set_of, ms, center, scale = sample_tables(11, S, per, n)
    flat = params(12)
    R = S * per
    per_epoch = R // B                     # 6: the replays below cross two passes
    steps = 8
    kw = dict(lr=3e-3, warmup=2, total=steps, lr_final=0.05, per_epoch=per_epoch)
    stream = torch.cuda.Stream()
    eager = nn.Surrogate(flat)
    graphed = nn.Surrogate(flat)
    perm_e = torch.empty(per_epoch * B, dtype=torch.int64, device="cuda:0")
    perm_g = torch.empty_like(perm_e)
    sch_e = nn.sched(**kw)
    sch_g = nn.sched(**kw)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        graph = graphed.capture_step(feat, pos, set_of, ms, center, scale, perm_g, sch_g, B, stream=stream)
        rng_e, rng_g = np.random.default_rng(5), np.random.default_rng(5)
        for step in range(1, steps + 1):
            say(f"graph replay step={step}")
            if (step - 1) % per_epoch == 0:
                perm_e.copy_(torch.from_numpy(rng_e.permutation(R)[:per_epoch * B].astype(np.int64)))
                perm_g.copy_(torch.from_numpy(rng_g.permutation(R)[:per_epoch * B].astype(np.int64)))
            x, t = eager.batch(feat, pos, set_of, ms, center, scale, perm_e, sch_e, B, stream=stream)
            loss_e = eager.train_step(x, t, sch_e, stream=stream)
            graph.launch(stream)
            stream.synchronize()
            assert torch.equal(graph.x, x) and torch.equal(graph.t, t), step
            assert float(loss_e.cpu()[0]) == float(graph.loss.cpu()[0]), step
            assert_same(state_of(eager), state_of(graphed), f"replay {step}")
    assert nn.sched_read(sch_g)["step"] == steps == nn.sched_read(sch_e)["step"]
    graph.close()


def test_captured_training_reduces_loss():
    """A short captured run on a learnable target (makespan proportional to the
    position of kernel 0) brings the loss down."""
    S, per, n, B = 2, 512, 8, 128
    feat, pos, set_of, _, center, scale = sample_tables(13, S, per, n)
    p = pos.cpu().numpy().astype(np.int64)
    ms = torch.from_numpy(10_000 + 100 * np.minimum(p[:, 0], n)).to("cuda:0")
    center = torch.full((S,), 10_000, dtype=torch.int64, device="cuda:0")
    scale = torch.full((S,), 400, dtype=torch.int64, device="cuda:0")
    model = nn.Surrogate(params(14, scale=0.05))
    per_epoch = (S * per) // B
    steps = 120
    sch = nn.sched(lr=3e-3, warmup=10, total=steps, lr_final=0.05, per_epoch=per_epoch)
    perm = torch.empty(per_epoch * B, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(0)
    torch.cuda.synchronize()
    losses = []
    with torch.cuda.stream(stream):
        graph = model.capture_step(feat, pos, set_of, ms, center, scale, perm, sch, B, stream=stream)
        for step in range(1, steps + 1):
            if (step - 1) % per_epoch == 0:
                perm.copy_(torch.from_numpy(rng.permutation(S * per)[:per_epoch * B].astype(np.int64)))
            graph.launch(stream)
            if step in (1, steps):
                losses.append(float(graph.loss.cpu()[0]))
    stream.synchronize()
    say(f"captured training loss {losses[0]:.4f} -> {losses[1]:.4f}")
    assert losses[1] < 0.5 * losses[0], losses
    graph.close()
