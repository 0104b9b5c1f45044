"""GPU parity of the depth-order network's pieces against the CPU oracle: canonical features
(bit-exact), meet-in-the-middle labels (against brute force), parameter init (bit-exact),
gradients of the BF16/MFMA path (tolerance from BF16 rounding), training and the depth order."""

import numpy as np
import pytest

import seeded_inputs
from oracle import bfs
from oracle import mlp as omlp
from oracle import zmat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_07413_amd import tcw
    assert torch.cuda.is_available()
    return tcw.Context(0)


def oracle_target(n, k, seed, clifford=None):
    tw = seeded_inputs.target_words(n, k, seed)
    cl = tw.clifford if clifford is None else clifford
    return tw, zmat.target_from_words(n, tw.paulis, cl)


@pytest.mark.parametrize("n,k,seed", [(1, 4, 1), (2, 3, 2), (2, 6, 3), (3, 5, 4), (3, 7, 5)])
def test_features_bit_exact(ctx, n, k, seed):
    import torch
    print("features", n, k, seed, flush=True)
    tw, u = oracle_target(n, k, seed)
    tgt = ctx.target_from_words(n, tw.paulis, tw.clifford)
    out = torch.empty(16 ** n, dtype=torch.float32, device="cuda:0")
    ctx.features(tgt, out)
    want = omlp.features(u)
    got = out.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_features_left_clifford_invariant(ctx):
    import torch
    tw, u = oracle_target(3, 5, 9)
    other = seeded_inputs.random_clifford_word(3, 77)
    t1 = ctx.target_from_words(3, tw.paulis, tw.clifford)
    t2 = ctx.target_from_words(3, tw.paulis, other)
    a = torch.empty(4096, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    ctx.features(t1, a)
    ctx.features(t2, b)
    assert torch.equal(a, b)


def _label(ctx, n, words, h_max, seed=11):
    import torch
    feats = torch.empty((len(words), 16 ** n), dtype=torch.float32, device="cuda:0")
    labels = torch.empty(len(words), dtype=torch.int32, device="cuda:0")
    ctx.label_batch(n, words, h_max, seed, feats, labels)
    return feats, labels.cpu().tolist()


def test_labels_match_brute_force_n1(ctx):
    print("labels n1", flush=True)
    _, seen, _ = bfs.cosets_by_tcount(1, 6)
    words, us = [], []
    for seed in range(40):
        k = 1 + seed % 8
        tw, u = oracle_target(1, k, seed)
        words.append((tw.paulis, tw.clifford))
        us.append(u)
    feats, labels = _label(ctx, 1, words, 3)
    for u, lab in zip(us, labels):
        t = bfs.min_tcount(u, seen)
        assert lab == (t if t is not None else -1)
    # features from the batch kernel equal the single-target ones
    assert np.array_equal(feats[0].cpu().numpy(), omlp.features(us[0]))


def test_labels_match_brute_force_n2(ctx):
    print("labels n2", flush=True)
    _, seen, _ = bfs.cosets_by_tcount(2, 3)
    words, us = [], []
    for seed in range(24):
        k = 1 + seed % 4
        tw, u = oracle_target(2, k, 50 + seed)
        words.append((tw.paulis, tw.clifford))
        us.append(u)
    _, labels = _label(ctx, 2, words, 2)
    for u, lab in zip(us, labels):
        t = bfs.min_tcount(u, seen)
        if t is not None:
            assert lab == t
        else:
            assert lab == 4   # T-count 4 (<= generating k = 4, not in levels 0..3)


def test_labels_n3_consistent(ctx):
    """n = 3: labels are at most the generating k, equal across left Cliffords, and match the
    exhaustive search for T-count <= 5 (depths <= 5 are enumerated)."""
    from paper_1606_07413_amd import tcw
    print("labels n3", flush=True)
    words, specs = [], []
    for seed in range(8):
        k = 2 + seed % 5
        tw = seeded_inputs.target_words(3, k, 400 + seed)
        words.append((tw.paulis, tw.clifford))
        words.append((tw.paulis, seeded_inputs.random_clifford_word(3, 900 + seed)))
        specs.append((k, tw))
    _, labels = _label(ctx, 3, words, 3)
    for i, (k, tw) in enumerate(specs):
        a, b = labels[2 * i], labels[2 * i + 1]
        assert a == b and 0 <= a <= k
        if k <= 5:
            tgt = ctx.target_from_words(3, tw.paulis, tw.clifford)
            p = ctx.default_params(3)
            p.k_max = 5
            res = ctx.search(tgt, p)
            assert res.status == 1 and res.t == a


def test_labels_n3_batch_split(ctx):
    """n = 3, a batch of 256: large enough that the labeller tables identity-side cosets up to T-count 4
    and probes at most 2 rotations per target.  Its labels equal the one-target certificate's, which
    keeps the balanced 3 + 3 split, and the exhaustive search's for small generating k."""
    print("labels n3 batch split", flush=True)
    words, tws = [], []
    for seed in range(256):
        k = 1 + seed % 10
        tw = seeded_inputs.target_words(3, k, 7000 + seed)
        words.append((tw.paulis, tw.clifford))
        tws.append((k, tw))
    _, labels = _label(ctx, 3, words, 3)
    seen = set()
    for i in range(0, 200, 3):      # every generating k in 1..10
        k, tw = tws[i]
        tgt = ctx.target_from_words(3, tw.paulis, tw.clifford)
        want = ctx.min_tcount(tgt, 3)
        assert labels[i] == want, (i, k)
        assert labels[i] <= k
        if 2 <= k <= 4:
            p = ctx.default_params(3)
            p.k_max = 4
            res = ctx.search(tgt, p)
            assert res.status == 1 and res.t == labels[i]
        tgt.free()
        seen.add(labels[i])
    # T-counts that need 0, 1 and 2 target-side rotations, and some beyond 6, are all covered
    assert {3, 4, 5, 6, -1} <= seen


def test_init_bit_exact(ctx):
    from paper_1606_07413_amd import tcw
    net = tcw.Network(ctx, 256, 64, 3, 11, seed=42)
    want = tcw.flatten_params(seeded_inputs.mlp_init(256, 64, 3, 11, 42), 3)
    assert np.array_equal(net.params(), want)


U_BF16 = 2.0 ** -8     # unit roundoff of bfloat16 (8 significant bits, round to nearest even)
U_F32 = 2.0 ** -24     # unit roundoff of float32
GELU1 = 1.1289         # max |gelu'|
GELU2 = 0.7979         # max |gelu''| (2 / sqrt(2 pi), at 0)


def _gam(m):
    """gamma_m = m u / (1 - m u): bound on the relative error of an m-term float32 sum of products."""
    return m * U_F32 / (1.0 - m * U_F32)


def gradient_error_bounds(params, x, labels, depth, u_bf16=U_BF16):
    """Elementwise first-order bounds on |GPU - oracle| for every gradient and probability of the
    network, from the GPU's arithmetic: BF16 operands that are exact in FP32 products, FP32
    accumulation over K terms (|error| <= gamma_K sum |a b|), FP32 GELU / softmax evaluation (a few
    FP32 ulps), and the rounding of every stored activation H and back-propagated G to BF16
    (relative error <= 2^-8).  The oracle's values are in float64 on the same BF16-rounded weights and
    inputs.  A running error analysis (Higham, Accuracy and Stability of Numerical Algorithms, Ch. 3):
    each bound is propagated through the next product by |.| matrices.  With u_bf16 = 0 it bounds the
    FP32 part alone."""
    from oracle import mlp as omlp
    b = x.shape[0]
    W = [params[f"W{l}"].astype(np.float64) for l in range(depth + 1)]
    bias = [params[f"b{l}"].astype(np.float64) for l in range(depth + 1)]
    absW = [np.abs(w) for w in W]
    logits, cache = omlp.forward(params, x, depth)
    h = [cache["h0"]] + [cache[f"h{l + 1}"] for l in range(depth)]
    z = [cache[f"z{l}"] for l in range(depth)]
    Eh = [np.zeros_like(h[0])]
    Ez = []
    for l in range(depth):
        K = W[l].shape[0]
        ez = Eh[l] @ absW[l] + _gam(K + 1) * ((np.abs(h[l]) + Eh[l]) @ absW[l] + np.abs(bias[l]))
        d = GELU1 * ez + 8 * U_F32 * (np.abs(z[l]) + ez + 1.0)         # FP32 gelu of the perturbed input
        Ez.append(ez)
        Eh.append(u_bf16 * np.abs(h[l + 1]) + (1 + u_bf16) * d)       # stored as BF16
    K = W[depth].shape[0]
    ezL = Eh[depth] @ absW[depth] + _gam(K + 1) * ((np.abs(h[depth]) + Eh[depth]) @ absW[depth]
                                                   + np.abs(bias[depth]))
    p = omlp.softmax(logits)
    Ep = p * (ezL + (p * ezL).sum(axis=1, keepdims=True)) + 32 * U_F32 * p
    g = p.copy()
    g[np.arange(b), labels] -= 1.0
    g /= b
    Eg = Ep / b + U_F32 * np.abs(g)                                      # FP32 G of the output layer
    bounds = {}
    for l in range(depth, -1, -1):
        Egb = u_bf16 * np.abs(g) + (1 + u_bf16) * Eg                   # G as BF16 for the products
        aH, aG = np.abs(h[l]) + Eh[l], np.abs(g) + Egb
        bounds[f"W{l}"] = np.abs(h[l]).T @ Egb + Eh[l].T @ aG + _gam(b + 16) * (aH.T @ aG)
        bounds[f"b{l}"] = Eg.sum(axis=0) + _gam(b) * np.abs(g).sum(axis=0)
        if l > 0:
            dh = g @ W[l].T
            Edh = Egb @ absW[l].T + _gam(W[l].shape[1]) * (aG @ absW[l].T)
            gp = omlp.gelu_grad(z[l - 1])
            Eg = (np.abs(dh) * (GELU2 * Ez[l - 1] + 8 * U_F32) + Edh * (np.abs(gp) + GELU2 * Ez[l - 1])
                  + U_F32 * np.abs(dh * gp))
            g = dh * gp
    return bounds, p, Ep


# Hoeffding: a sum of independent zero-mean terms with |X_k| <= c_k exceeds t with probability at most
# 2 exp(-2 t^2 / sum (2 c_k)^2); for rounding errors uniform in [-c_k, c_k] (variance c_k^2 / 3) and
# t = LAMBDA sigma that is 2 exp(-LAMBDA^2 / 6) < 1e-10 per element at LAMBDA = 12.
LAMBDA = 12.0


def gradient_error_sigmas(params, x, labels, depth):
    """Standard deviations of GPU - oracle under the probabilistic model of rounding errors (Higham and
    Mary, SIAM J. Sci. Comput. 2019): every rounding multiplies a value by (1 + d) with d independent,
    zero-mean and |d| <= u (variance u^2 / 3).  A BF16 store of an activation H or a back-propagated G
    (u = 2^-8) adds variance u^2 / 3 |value|^2; a K-term FP32 sum of products (u = 2^-24) adds at most
    K u^2 / 3 (sum |a b|)^2, every partial sum being bounded by the sum of absolute terms; FP32 GELU
    and softmax add a few FP32 ulps.  Variances propagate through each product by |.|^2 matrices."""
    from oracle import mlp as omlp
    ub = U_BF16 ** 2 / 3.0
    uf = U_F32 ** 2 / 3.0
    b = x.shape[0]
    W = [params[f"W{l}"].astype(np.float64) for l in range(depth + 1)]
    bias = [params[f"b{l}"].astype(np.float64) for l in range(depth + 1)]
    W2 = [w * w for w in W]
    aW = [np.abs(w) for w in W]
    logits, cache = omlp.forward(params, x, depth)
    h = [cache["h0"]] + [cache[f"h{l + 1}"] for l in range(depth)]
    z = [cache[f"z{l}"] for l in range(depth)]
    Vh = [np.zeros_like(h[0])]
    Vz = []
    for l in range(depth):
        K = W[l].shape[0]
        vz = Vh[l] @ W2[l] + (K + 1) * uf * (np.abs(h[l]) @ aW[l] + np.abs(bias[l])) ** 2
        Vz.append(vz)
        gp = omlp.gelu_grad(z[l])
        Vh.append(ub * h[l + 1] ** 2 + gp ** 2 * vz + 16 * uf * (np.abs(h[l + 1]) + np.abs(z[l] * gp) + 1e-30) ** 2)
    K = W[depth].shape[0]
    vzl = Vh[depth] @ W2[depth] + (K + 1) * uf * (np.abs(h[depth]) @ aW[depth] + np.abs(bias[depth])) ** 2
    p = omlp.softmax(logits)
    Vp = p ** 2 * (vzl + (p ** 2 * vzl).sum(axis=1, keepdims=True)) + 64 * uf * p ** 2
    g = p.copy()
    g[np.arange(b), labels] -= 1.0
    g /= b
    Vg = Vp / b ** 2 + uf * g ** 2
    sig = {}
    for l in range(depth, -1, -1):
        Vgb = ub * g ** 2 + Vg
        acc = (b + 16) * uf * (np.abs(h[l]).T @ np.abs(g)) ** 2
        sig[f"W{l}"] = np.sqrt((h[l] ** 2).T @ Vgb + Vh[l].T @ (g ** 2) + acc)
        sig[f"b{l}"] = np.sqrt(Vg.sum(axis=0) + b * uf * np.abs(g).sum(axis=0) ** 2)
        if l > 0:
            dh = g @ W[l].T
            vdh = Vgb @ W2[l].T + W[l].shape[1] * uf * (np.abs(g) @ aW[l].T) ** 2
            gp = omlp.gelu_grad(z[l - 1])
            Vg = gp ** 2 * vdh + (dh * GELU2) ** 2 * Vz[l - 1] + 16 * uf * (dh * gp) ** 2
            g = dh * gp
    return sig, np.sqrt(Vp)


# (inputs, hidden width, batch): the batch sizes from 1024 up split the weight-gradient reduction
# over several workgroups; the last case is the depth-order network's own shape (4096 -> 512 x 3 -> 11)
GRAD_CASES = [(256, 64, 37), (256, 64, 1024), (512, 128, 2048), (4096, 512, 4096)]


@pytest.mark.parametrize("inp,hidden,batch", GRAD_CASES)
def test_gradients_against_oracle(ctx, inp, hidden, batch):
    """Every gradient element and every probability of the BF16 MFMA path against the float64 oracle
    on the same BF16-rounded weights and inputs, within the running error bound of the GPU's
    arithmetic (gradient_error_bounds, doubled for second-order terms)."""
    import torch
    from paper_1606_07413_amd import tcw
    print("gradients", inp, hidden, batch, flush=True)
    depth, classes = 3, 11
    params = seeded_inputs.mlp_init(inp, hidden, depth, classes, 7)
    rng = np.random.default_rng(batch)
    for l in range(depth + 1):
        params[f"b{l}"] = (rng.normal(size=params[f"b{l}"].shape) * 0.05).astype(np.float32)
    x = rng.normal(size=(batch, inp)).astype(np.float32) * 0.5
    y = rng.integers(0, classes, batch).astype(np.int32)
    net = tcw.Network(ctx, inp, hidden, depth, classes, init=tcw.flatten_params(params, depth))
    xd = torch.tensor(x, device="cuda:0")
    g, loss = net.gradients(xd, torch.tensor(y, device="cuda:0"))
    probs = torch.empty((batch, classes), dtype=torch.float32, device="cuda:0")
    net.forward(xd, probs)
    # oracle on the BF16-rounded weights and inputs the GPU multiplies
    pr = {k: (omlp.bf16_round(v) if k.startswith("W") else v) for k, v in params.items()}
    xb = omlp.bf16_round(x).astype(np.float64)
    ref = omlp.gradients(pr, xb, y, depth)
    ref_loss = omlp.loss(pr, xb, y, depth)
    bounds, p_ref, p_bound = gradient_error_bounds(pr, xb, y, depth)
    sigmas, p_sigma = gradient_error_sigmas(pr, xb, y, depth)
    assert abs(loss - ref_loss) < 1e-2 * abs(ref_loss)
    err = np.abs(probs.cpu().numpy().astype(np.float64) - p_ref)
    assert np.all(err <= 2 * p_bound), float((err / p_bound).max())
    assert np.all(err <= 1e-2 * p_ref + LAMBDA * p_sigma), float((err / (p_sigma + 1e-30)).max())
    off = 0
    worst, worst_sigma = 0.0, 0.0
    for l in range(depth + 1):
        for name in (f"W{l}", f"b{l}"):
            size = params[name].size
            got = g[off:off + size].reshape(params[name].shape).astype(np.float64)
            off += size
            e = np.abs(got - ref[name])
            # rigorous: the worst-case running bound (doubled for second-order terms)
            worst = max(worst, float((e / np.maximum(bounds[name], 1e-30)).max()))
            assert np.all(e <= 2 * bounds[name]), (name, float((e / bounds[name]).max()))
            # tight: 1e-2 relative plus LAMBDA standard deviations of the rounding model
            tol = 1e-2 * np.abs(ref[name]) + LAMBDA * sigmas[name]
            worst_sigma = max(worst_sigma, float((e / tol).max()))
            assert np.all(e <= tol), (name, float((e / tol).max()))
    print("largest error / worst-case bound", worst, "largest error / tolerance", worst_sigma, flush=True)


def test_forward_probs(ctx):
    import torch
    from paper_1606_07413_amd import tcw
    net = tcw.Network(ctx, 256, 64, 3, 11, seed=5)
    x = torch.randn((50, 256), device="cuda:0")
    p = torch.empty((50, 11), device="cuda:0")
    net.forward(x, p)
    assert torch.allclose(p.sum(dim=1), torch.ones(50, device="cuda:0"), atol=1e-5)


def test_training_reduces_loss_and_orders_depths(ctx):
    """n = 2 targets with k uniform in 1..6, labelled exactly (h_max = 3): training lowers the
    loss; the depth order is a permutation led by the most probable T-count."""
    import torch
    from paper_1606_07413_amd import tcw
    print("train n2", flush=True)
    words = []
    for seed in range(2048):
        tw = seeded_inputs.target_words(2, 1 + seed % 6, 10_000 + seed)
        words.append((tw.paulis, tw.clifford))
    feats, labels = _label(ctx, 2, words, 3)
    lab = torch.tensor(labels, dtype=torch.int32, device="cuda:0")
    assert (lab >= 0).all()
    net = tcw.Network(ctx, 256, 128, 3, 11, seed=42)
    first = net.train_step(feats, lab, 1e-3)
    for _ in range(60):
        last = net.train_step(feats, lab, 1e-3)
    assert last < 0.7 * first
    tw = seeded_inputs.target_words(2, 5, 77)
    order, probs = net.depth_order(ctx.target_from_words(2, tw.paulis, tw.clifford), 6)
    assert sorted(order) == list(range(7))
    assert probs[order[0]] == max(probs[:7])


def test_depth_costs_and_cost_aware_order(ctx):
    """tcw_depth_costs: a depth's cost is the steps the driver spends on it when it holds no
    decomposition (every chunk's budget beta N / theta, or its N points when enumerated, plus a fixed
    2^20); the cost-aware order sorts depths by p_k / c_k."""
    from paper_1606_07413_amd import tcw
    print("depth costs", flush=True)
    tw = seeded_inputs.target_words(3, 6, 5)
    tgt = ctx.target_from_words(3, tw.paulis, tw.clifford)
    p = ctx.default_params(3)
    p.k_max = 10
    p.log2_table = 24
    p.delta = -1
    costs = ctx.depth_costs(tgt, p, 10)
    fixed = float(1 << 20)
    assert costs[0] == fixed
    # depths 1..5: enumerated (N = 2 * 63^(k // 2) <= 2^16), 63 chunks at odd k
    assert costs[1] == fixed + 63 * 2
    assert costs[2] == fixed + 2 * 63
    assert costs[5] == fixed + 63 * 2 * 63 ** 2
    # depth 6: walks, N = 2 * 63^3, theta from the table: 8 N <= 2^(24 + delta) -> delta = 1
    n6 = 2 * 63 ** 3
    assert costs[6] == fixed + 16 * n6 * 2
    # depth 8: N = 2 * 63^4 -> delta = 4
    n8 = 2 * 63 ** 4
    assert costs[8] == fixed + 16 * n8 * 16
    assert all(costs[k] < costs[k + 2] for k in range(9))
    # a given delta and budget are used as given
    p.delta = 3
    p.budget_beta = 4
    assert ctx.depth_costs(tgt, p, 6)[6] == fixed + 4 * n6 * 8
    # order: depths by p_k / c_k (a network of untrained weights gives some p)
    net = tcw.Network(ctx, 4096, 64, 3, 11, seed=3)
    p.delta = -1
    p.budget_beta = 16
    order, probs = net.depth_order(tgt, 10, p)
    key = [probs[k] / costs[k] for k in range(11)]
    assert order == sorted(range(11), key=lambda k: (-key[k], k))
    order_p, _ = net.depth_order(tgt, 10)
    assert order_p == sorted(range(11), key=lambda k: (-probs[k], k))
    bad = ctx.default_params(3)
    bad.budget_beta = 0
    with pytest.raises(tcw.TcwError):
        ctx.depth_costs(tgt, bad, 6)
    with pytest.raises(tcw.TcwError):
        net.depth_order(tgt, 10, bad)


def test_learned_order_gains_over_plain(ctx):
    """A network trained on n = 3 circuits (k in 1..8; exact labels up to 6, the generating k above)
    orders depths by p_k / c_k.  On 64 held-out targets (k in 4..7), each searched alone, the first
    verified decomposition under that order (TCW_ORDER_GIVEN_FIRST) takes less wall time in total than
    the plain increasing order, which must fail every depth below the answer first (compared over the
    targets both orders solve with the minimal T-count).  Every learned answer is exact; one with a
    larger T-count than the plain order's is flagged not minimal.  The walk search is randomised, so
    either order can miss a decomposition within its budget: a few such misses are allowed and
    counted.  With the same order certified (TCW_ORDER_GIVEN) the answer is the minimum: for T-count
    <= 6 it equals the meet-in-the-middle certificate's."""
    import torch
    from oracle import search as osearch
    from paper_1606_07413_amd import tcw
    print("learned gain", flush=True)
    train = seeded_inputs.mlp_targets(20_000, 20_000 + 8192, k_lo=1, k_hi=8)
    feats, labels = _label(ctx, 3, [(w.paulis, w.clifford) for w in train], 3)
    lab = torch.tensor([v if v >= 0 else w.k for v, w in zip(labels, train)], dtype=torch.int32, device="cuda:0")
    net = tcw.Network(ctx, 4096, 256, 3, 11, seed=42)
    net.train(feats, lab, 512, 6, 1e-3)
    held = seeded_inputs.mlp_targets(30_000, 30_064, k_lo=4, k_hi=7)
    _, exact = _label(ctx, 3, [(w.paulis, w.clifford) for w in held], 3)
    secs = {"plain": 0.0, "learned": 0.0}
    misses = {"plain": 0, "learned": 0}
    larger = compared = 0
    for i, w in enumerate(held):
        tgt = ctx.target_from_words(3, w.paulis, w.clifford)
        found = {}
        for name in ("plain", "learned", "certified"):
            if name == "certified" and i % 4:
                continue
            p = ctx.default_params(3)
            p.k_max = 8
            p.seed = 40 + i
            p.log2_table = 22
            p.chunk_parallel = 0
            p.max_seconds = 5.0
            if name != "plain":
                order, _ = net.depth_order(tgt, 8, p)
                p.depth_order_kind = tcw.ORDER_GIVEN_FIRST if name == "learned" else tcw.ORDER_GIVEN
                p.depth_order_len = len(order)
                for j, kk in enumerate(order):
                    p.depth_order[j] = kk
            found[name] = ctx.search(tgt, p)
        u = zmat.target_from_words(3, w.paulis, w.clifford)
        for name, r in found.items():
            if r.status == 1:
                d = tcw.decomposition_of(r)
                assert osearch.reconstruct(3, osearch.Decomposition(t=d.t, paulis_desc=d.paulis_desc, perm=d.perm,
                                                                    sign=d.sign)).equals(u), (i, name)
                if exact[i] >= 0:
                    assert r.t >= exact[i]
                    assert r.minimal == 0 or r.t == exact[i], (i, name)
            elif name in misses:
                misses[name] += 1
        pl, le = found["plain"], found["learned"]
        if pl.status == 1 and exact[i] >= 0:
            assert pl.t == exact[i] and pl.minimal == 1
        if pl.status == 1 and le.status == 1:
            if le.t > pl.t:
                assert le.minimal == 0
                larger += 1
            else:
                assert le.t == pl.t
                secs["plain"] += pl.seconds
                secs["learned"] += le.seconds
                compared += 1
        if "certified" in found and found["certified"].status == 1:
            ce = found["certified"]
            assert ce.minimal == 1
            if exact[i] >= 0:
                assert ce.t == exact[i] == ctx.min_tcount(tgt, 3)
        tgt.free()
    print("total seconds", secs, "over", compared, "targets; misses", misses, "larger T-count", larger, flush=True)
    assert misses["plain"] <= 2 and misses["learned"] <= 2 and larger <= 2
    assert compared >= 58
    assert secs["learned"] < secs["plain"]


def test_label_batch_validates_words(ctx):
    """Word arrays that do not describe valid words are refused on the host, before the device reads
    them: a Pauli code out of range, kof above the word length, decreasing offsets, an over-long word."""
    import ctypes
    import torch
    from paper_1606_07413_amd import tcw
    n = 2
    feats = torch.empty((1, 16 ** n), dtype=torch.float32, device="cuda:0")
    labels = torch.empty(1, dtype=torch.int32, device="cuda:0")

    def call(words, offsets, kof):
        w = (ctypes.c_uint16 * max(1, len(words)))(*words)
        o = (ctypes.c_int32 * len(offsets))(*offsets)
        k = (ctypes.c_int32 * len(kof))(*kof)
        return ctx.lib.tcw_label_batch(ctx.h, n, len(kof), w, o, k, 2, 5, feats.data_ptr(), labels.data_ptr())

    assert call([3, 5, 7], [0, 3], [2]) == 0
    assert call([3, 16, 7], [0, 3], [2]) == tcw.TCW_EINVAL       # code above 4^n - 1
    assert call([3, 0, 7], [0, 3], [2]) == tcw.TCW_EINVAL        # the identity
    assert call([3, 5, 7], [0, 3], [4]) == tcw.TCW_EINVAL        # kof above the word length
    assert call([3, 5, 7], [1, 3], [1]) == tcw.TCW_EINVAL        # offsets[0] != 0
    assert call([3] * 200, [0, 200], [10]) == tcw.TCW_EINVAL     # 2 * 190 + 10 rotations

