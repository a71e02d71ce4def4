"""GPU parity of the warm-start network (BF16 MFMA kernels) against the FP64
reference in oracle/mlp.py, and the warm start's effect on the iteration.

Tolerances.  Weights are the same BF16 values on both sides and the inputs
are exactly +-1, so the only differences are the FP32 accumulation order of
the matrix cores against exact FP64 sums (relative 2^-24 per operation), and
the rare BF16 rounding of an activation that lands on the other side of a
rounding boundary because of that (one BF16 step, relative 2^-8, for that
activation).  The forward check therefore asks for agreement to 1e-4 of the
output scale on 99% of samples and to 2^-5 of the scale on all; the backward
also rounds every upstream gradient to BF16 (relative 2^-9 each): against
the oracle's backward with the same rounding points every gradient entry is
checked element by element (test_backward_matches_reference_element_by_element
states the bound), and against the exact FP64 gradient each tensor must agree
to 2e-2 in relative L2 norm with cosine >= 0.999.
"""
import sys

import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2407_10925_amd as pk
    return pk


def _params(seed, scale=0.1):
    u = si.uniform(seed, torch.arange(omlp.NPARAMS, dtype=torch.int64), scale=2.0)  # [0, 2)
    return ((u - 1.0) * scale).to(torch.float32)


def _indices(n, count, seed):
    return si.sample_indices(n, count, seed)[:count]


def test_to_bf16_bit_exact(pk):
    say("bf16 conversion")
    p = _params(1, scale=3.0)
    M = pk.Mlp(batch=256)
    M.load(p.cuda())
    got = M.wbf16.cpu().numpy().view(np.uint16)
    ref = omlp.bf16(p.numpy().astype(np.float64)).astype(np.float32).view(np.uint32) >> 16
    assert np.array_equal(got.astype(np.uint32), ref)


def test_init_is_seeded_and_scaled(pk):
    a = pk.Mlp(seed=5, batch=256).params.cpu().numpy()
    b = pk.Mlp(seed=5, batch=256).params.cpu().numpy()
    c = pk.Mlp(seed=6, batch=256).params.cpu().numpy()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    P = omlp.unpack(a)
    assert np.all(P["b1"] == 0) and np.all(P["b2"] == 0) and P["b4"][0] == 0
    assert np.max(np.abs(P["W1"])) <= np.sqrt(6 / 32) and np.max(np.abs(P["W2"])) <= np.sqrt(6 / 256)
    assert abs(np.std(P["W2"]) - np.sqrt(2 / 256)) < 0.1 * np.sqrt(2 / 256)


@pytest.mark.parametrize("h", [12, 16])
def test_forward_matches_reference(pk, h):
    say(f"forward h={h}")
    B = 1024
    p = _params(2)
    M = pk.Mlp(batch=B)
    M.load(p.cuda())
    idx = _indices(4 ** h, B, seed=7 + h)
    y = torch.empty(B, dtype=torch.float32, device="cuda")
    M.forward(idx.cuda(), h, y)
    got = y.cpu().numpy().astype(np.float64)
    ref, cache = omlp.forward(p.numpy().astype(np.float64), omlp.encode(idx.numpy().astype(np.uint64), h))
    scale = np.abs(cache["a3"]) @ np.abs(cache["w4"]) + abs(float(p[-1])) + 1e-3
    err = np.abs(got - ref) / scale
    say(f"forward max rel err {err.max():.2e}, 99th pct {np.quantile(err, 0.99):.2e}")
    assert np.quantile(err, 0.99) <= 1e-4
    assert err.max() <= 2.0 ** -5


def _gradient_magnitudes(cache, dy):
    """For every gradient entry, the sum of the absolute values of the terms
    it sums: |dZ_k|^T |a_(k-1)| for the weights of layer k (a_0 = the
    inputs), sum_s |dZ_k| for its biases, |a_3|^T |dy| and sum_s |dy| for the
    output layer (dZ_k and a_k as the oracle's backward with the GPU's
    rounding points produces them; dy may carry an allowance for the forward
    error, see the test)."""
    A = {"W1": np.abs(cache["X"]), "W2": np.abs(cache["a1"]), "W3": np.abs(cache["a2"])}
    D = {"W1": np.abs(cache["dz1"]), "W2": np.abs(cache["dz2"]), "W3": np.abs(cache["dz3"])}
    m = {k: D[k].T @ A[k] for k in A}
    m.update({"b1": D["W1"].sum(0), "b2": D["W2"].sum(0), "b3": D["W3"].sum(0),
              "w4": np.abs(cache["a3"]).T @ np.abs(dy), "b4": np.array([np.abs(dy).sum()])})
    out = np.empty(omlp.NPARAMS)
    for k, (o, shp) in omlp.OFFSETS.items():
        out[o:o + int(np.prod(shp))] = m[k].reshape(-1)
    return out


def test_backward_matches_reference_element_by_element(pk):
    """Every gradient entry against the oracle's backward with the GPU's
    rounding points (bf16_grads).  Both sides round the same quantities to
    BF16 and differ only by FP32 accumulation (relative 2^-24 per addition)
    and by the rare value that this moves across a BF16 rounding boundary (one
    BF16 step, at most 2^-7 of it): so each entry must lie within 2^-7 of the
    sum of the absolute values of its terms (every term off by one step), and
    all but 0.1% within 2^-12 of it.  (An FP32 emulation of the same steps on
    the CPU stays within 4e-5 of that sum.)  The output layer's gradient
    multiplies by dy, which inherits the forward's error; its terms carry
    that error's bound too, and only the first criterion applies there."""
    say("backward, element by element")
    B, h = 512, 12
    p = _params(3)
    M = pk.Mlp(batch=B)
    M.load(p.cuda())
    idx = _indices(4 ** h, B, seed=11)
    t = si.uniform(12, torch.arange(B), scale=4.0).to(torch.float32)
    y = torch.empty(B, dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    idx_d = idx.cuda()
    M.forward(idx_d, h, y, keep=True)
    M.loss(y, t.cuda(), dy)
    M.backward(idx_d, h, dy)
    g = M.grad.cpu().numpy().astype(np.float64)
    p64 = p.numpy().astype(np.float64)
    yr, cache = omlp.forward(p64, omlp.encode(idx.numpy().astype(np.uint64), h))
    _, dy_r = omlp.mse(yr, t.numpy())
    gr = omlp.backward(cache, dy_r, bf16_grads=True)
    # dy = 2 (y - t) / B comes from the forward, whose output the GPU computes
    # within 2^-5 of its scale (test_forward_matches_reference): where y is
    # close to t that is a large part of dy itself, so the output layer's
    # terms carry that allowance beside their own value
    scale = np.abs(cache["a3"]) @ np.abs(cache["w4"]) + abs(float(p[-1])) + 1e-3
    edy = 2.0 * 2.0 ** -5 * scale / B
    mag = _gradient_magnitudes(cache, dy_r)
    out_layer = _gradient_magnitudes(cache, np.abs(dy_r) + edy)
    for k in ("w4", "b4"):
        o, shape = omlp.OFFSETS[k]
        n = int(np.prod(shape))
        mag[o:o + n] = out_layer[o:o + n]
    for name, (o, shape) in omlp.OFFSETS.items():
        n = int(np.prod(shape))
        diff, m = np.abs(g[o:o + n] - gr[o:o + n]), mag[o:o + n]
        r = diff / np.maximum(m, 1e-300)
        say(f"grad {name}: max |diff| / sum|terms| {r.max():.2e}, 99.9th pct "
            f"{np.quantile(r, 0.999):.2e}")
        assert np.all(diff <= 2.0 ** -7 * m + 1e-30), name
        if name not in ("w4", "b4"):  # their spread is the forward's, bounded above
            assert np.quantile(r, 0.999) <= 2.0 ** -12, name


def test_backward_matches_reference_in_norm(pk):
    """A second, coarser view: per tensor against the exact FP64 gradient,
    relative L2 error and cosine."""
    say("backward")
    B, h = 512, 12
    p = _params(3)
    M = pk.Mlp(batch=B)
    M.load(p.cuda())
    idx = _indices(4 ** h, B, seed=11)
    t = si.uniform(12, torch.arange(B), scale=4.0).to(torch.float32)
    y = torch.empty(B, dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    idx_d = idx.cuda()
    M.forward(idx_d, h, y, keep=True)
    M.loss(y, t.cuda(), dy)
    M.backward(idx_d, h, dy)
    g = M.grad.cpu().numpy().astype(np.float64)
    yr, cache = omlp.forward(p.numpy().astype(np.float64), omlp.encode(idx.numpy().astype(np.uint64), h))
    loss_r, dy_r = omlp.mse(yr, t.numpy())
    assert abs(M.loss_dev.item() - loss_r) <= 1e-3 * loss_r
    gr = omlp.backward(cache, dy_r)
    for name, (o, shape) in omlp.OFFSETS.items():
        n = int(np.prod(shape))
        a, b = g[o:o + n], gr[o:o + n]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        say(f"grad {name}: rel {rel:.2e} cos {cos:.6f}")
        assert rel <= 2e-2 and cos >= 0.999, name


def test_adam_step_matches_reference(pk):
    M = pk.Mlp(batch=256)
    p = _params(4)
    g = _params(5, scale=1e-2)
    M.load(p.cuda())
    M.grad.copy_(g.cuda())
    M.adam(1e-3)
    M.grad.copy_((g * 0.5).cuda())
    M.adam(1e-3)
    q, m, v = omlp.adam(p.numpy().astype(np.float64), g.numpy().astype(np.float64),
                        np.zeros(omlp.NPARAMS), np.zeros(omlp.NPARAMS), 1, 1e-3)
    q, m, v = omlp.adam(q, 0.5 * g.numpy().astype(np.float64), m, v, 2, 1e-3)
    np.testing.assert_allclose(M.params.cpu().numpy(), q, rtol=0, atol=2e-6)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sample_draws_in_range_and_gathers_targets(pk, dtype):
    """Sampling from a folded table (the 4^h / 2 stored entries) gathers the
    value of every drawn index, also those read at their complement."""
    h = 9
    full = si.table(2, 2, h, seed=33, dtype=dtype)
    table = full[:4 ** h // 2].cuda()
    M = pk.Mlp(batch=4096)
    M.sample(table, h, seed=1)
    idx = M.idx.cpu().numpy()
    assert idx.min() >= 0 and idx.max() < 4 ** h
    assert len(np.unique(idx)) > 3000 and (idx >= 4 ** h // 2).sum() > 1000
    tab = full.numpy().astype(np.float64)
    assert np.array_equal(M.target.cpu().numpy(), (tab[idx] - tab[0]).astype(np.float32))


def _converged_table(pk, h, sweeps):
    L = pk.Lcsb(2, 2, h, "f64")
    L.init_zero()
    L.iterate(sweeps)
    _, best = L.certify()
    return L, best


def _swap_strings(i):
    """Index of the same tuple with strings a and b exchanged (pair layout)."""
    ev = 0x5555555555555555
    return ((i >> 1) & ev) | ((i & ev) << 1)


def test_training_reduces_the_loss_and_seed_is_consistent(pk):
    """Train on a converged l = 8 table; the loss falls by 10x.  Seed an
    l = 8 ring that was filled with NaN: every entry is written, lag 2 is
    invariant under exchanging the strings and under complementing both,
    each lag 2 value is the network's output at one member of that orbit,
    and lag 1 = lag 2 + rate."""
    say("training on l=8")
    h = 8
    L, best = _converged_table(pk, h, 160)
    table, _ = L.lag(1)
    M = pk.Mlp(batch=1024, seed=9)
    losses = []
    for step in range(300):
        M.train_step(table, h, seed=1000 + step, lr=2e-3)
        if step % 50 == 0 or step == 299:
            losses.append(M.loss_dev.item())
    say(f"losses {losses}")
    assert losses[-1] < losses[0] / 10
    R = L.certify()[0]["R"]
    n = 4 ** h
    S = pk.Lcsb(2, 2, h, "f32")
    nan = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    S.load_ring([nan, nan.clone()])
    S.init_seed_mlp(M, rate=R)
    assert S.swap_symmetric()  # one value per exchange orbit: sweeps run folded
    lag2 = S.lag(2)[0].cpu()
    lag1 = S.lag(1)[0].cpu()
    assert lag2.numel() == n // 2
    assert not torch.isnan(lag2).any() and not torch.isnan(lag1).any()
    i = np.arange(n, dtype=np.uint64)
    j = _swap_strings(i)
    m = np.uint64(n - 1)
    stored = si.representative(torch.arange(n, dtype=torch.int64), 2, 2, h).numpy()
    l2 = lag2.numpy()[stored]  # every index, read at its stored representative
    assert np.array_equal(l2, l2[j.astype(np.int64)])
    assert np.array_equal(l2, l2[(i ^ m).astype(np.int64)])
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    M.forward(torch.arange(n, dtype=torch.int64, device="cuda"), h, y)
    yh = y.cpu().numpy()
    members = [i, j, i ^ m, j ^ m]
    hit = np.zeros(n, dtype=bool)
    for mem in members:
        hit |= l2 == yh[mem.astype(np.int64)]
    assert hit.all()
    assert torch.equal(lag1, (lag2.double() + R).float())


def _sweeps_to_gap(S, target, gap, limit=300):
    """FP32 sweeps (a certificate every 2) until the best bound is within gap of target."""
    while True:
        S.iterate(2)
        _, best = S.certify()
        if target - best["bound"] <= gap or best["sweep"] >= limit:
            return best["sweep"], best


def test_seeded_run_gains_sweeps_and_reaches_the_plain_bound(pk):
    """l = 10: the network trained on converged l = 8 and l = 9 tables seeds
    an FP32 ring.  What the network gains over the method without it: the
    seeded FP32 run comes within 1e-5 of the plain FP64 bound in fewer sweeps
    than the zero-started one.  The seeded run then reaches the plain bound
    within 1e-9 after the FP64 polish (the limit does not depend on the
    start)."""
    say("seeded run l=10")
    P, plain = _converged_table(pk, 10, 240)
    B = plain["bound"]
    M = pk.Mlp(batch=2048, seed=10)
    tabs = []
    for h in (8, 9):
        L, _ = _converged_table(pk, h, 200)
        tabs.append((h, L))
    tables = [(h, L.lag(1)[0]) for h, L in tabs]
    for step in range(400):
        h, table = tables[step % 2]
        M.train_step(table, h, seed=step, lr=2e-3)
    rate = tabs[1][1].certify()[0]["R"]
    Z = pk.Lcsb(2, 2, 10, "f32")
    Z.init_zero()
    zero_sweeps, _ = _sweeps_to_gap(Z, B, 1e-5)
    S = pk.Lcsb(2, 2, 10, "f32")
    S.init_seed_mlp(M, rate=rate)
    seeded_sweeps, best = _sweeps_to_gap(S, B, 1e-5)
    say(f"sweeps to within 1e-5 of the plain bound: zero start {zero_sweeps}, seeded {seeded_sweeps}")
    assert B - best["bound"] <= 1e-5
    assert seeded_sweeps < zero_sweeps
    Q = pk.Lcsb(2, 2, 10, "f64")
    Q.upcast(S)
    for _ in range(40):
        Q.iterate(4)
        _, best = Q.certify()
        if best["bound"] >= B - 1e-9:
            break
    say(f"seeded {best['bound']:.12f} at sweep {best['sweep']}, plain {B:.12f}")
    assert abs(best["bound"] - B) <= 1e-9


def test_seed_at_l16_matches_the_oracle_network(pk):
    """The l = 16 seed, computed by the orbit-enumerating forward kernel that
    the time-to-bound runs use, against the oracle's forward: at 4000 sampled
    stored entries, lag 2 is the network's output at one member of the
    entry's orbit (exchange of the strings, complement of both) within the
    forward tolerance, and lag 1 = lag 2 + rate."""
    h = 16
    n = 4 ** h
    free, _ = torch.cuda.mem_get_info()
    if free < 24 * 2 ** 30:
        pytest.skip("needs 24 GiB of free device memory")
    say("seed at l=16 against the oracle network")
    p = _params(21)
    M = pk.Mlp(batch=256)
    M.load(p.cuda())
    rate = 0.39
    S = pk.Lcsb(2, 2, h, "f32")
    S.init_seed_mlp(M, rate=rate)
    idx = si.sample_indices(n // 2, 4000, seed=17)
    lag2 = S.lag(2)[0][idx.cuda()].cpu()
    lag1 = S.lag(1)[0][idx.cuda()].cpu()
    del S
    torch.cuda.empty_cache()
    assert torch.equal(lag1, (lag2.double() + rate).float())
    i = idx.numpy().astype(np.uint64)
    j = np.array([_swap_strings(int(v)) for v in i], dtype=np.uint64)
    full = np.uint64(n - 1)
    p64 = p.numpy().astype(np.float64)
    outs, scales = [], []
    for mem in (i, j, i ^ full, j ^ full):
        y, cache = omlp.forward(p64, omlp.encode(mem, h))
        outs.append(y)
        scales.append(np.abs(cache["a3"]) @ np.abs(cache["w4"]) + abs(float(p[-1])) + 1e-3)
    scale = np.max(np.stack(scales), axis=0)
    err = np.min(np.abs(np.stack(outs) - lag2.numpy().astype(np.float64)[None, :]), axis=0) / scale
    say(f"seed vs oracle: max rel err {err.max():.2e}, 99th pct {np.quantile(err, 0.99):.2e}")
    assert np.quantile(err, 0.99) <= 1e-4
    assert err.max() <= 2.0 ** -5
