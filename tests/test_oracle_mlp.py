"""Pins of the oracle's monotone MLP (learned-partition extension): analytic
gradient against central finite differences, closed forms of the quantile
initialisation and of tiny networks, monotonicity, and the defining property
of the bucket thresholds."""
import numpy as np
import pytest

import oracle
import synth

U64 = 2**64 - 1


def random_params(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    p = np.zeros(oracle.MLP_NP, dtype=np.float32)
    p[oracle.W1:oracle.W1 + 32] = rng.uniform(0.5, 3.0, 32)
    p[oracle.B1:oracle.B1 + 32] = rng.uniform(-1.5, 0.5, 32)
    p[oracle.W2:oracle.W2 + 1024] = rng.uniform(0.0, scale / 8, 1024)
    p[oracle.B2:oracle.B2 + 32] = rng.uniform(-0.2, 0.4, 32)
    p[oracle.W3:oracle.W3 + 32] = rng.uniform(0.0, 0.06, 32)
    p[oracle.B3] = 0.01
    return p


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = random_params(1)
    u = rng.uniform(0, 1, 200)
    y = np.sort(rng.uniform(0, 1, 200))
    loss, g = oracle.mlp_loss_grad(p, u, y)
    # the loss is evaluated in float64 from float32 parameters: perturb by a
    # small exact float32 step (so that no clamp kink is crossed) and divide
    # by the step actually taken
    checked = 0
    for idx in list(range(0, 64, 7)) + list(range(64, 1088, 97)) + list(range(1088, 1153, 5)):
        h = np.float32(2.0**-18) * max(np.float32(1e-2), abs(p[idx]))
        pp, pm = p.copy(), p.copy()
        pp[idx] += h
        pm[idx] -= h
        hp = float(pp[idx]) - float(p[idx])
        hm = float(p[idx]) - float(pm[idx])
        lp, _ = oracle.mlp_loss_grad(pp, u, y)
        lm, _ = oracle.mlp_loss_grad(pm, u, y)
        fd = (lp - lm) / (hp + hm)
        assert abs(fd - g[idx]) <= 1e-4 * abs(g[idx]) + 1e-9, (idx, fd, g[idx])
        checked += 1
    assert checked > 20


def test_gradient_zero_at_perfect_fit_and_sign():
    """identity network f(u) = u on targets y = u: zero loss, zero gradient;
    raising the output bias raises the loss with a positive derivative."""
    p = np.zeros(oracle.MLP_NP, dtype=np.float32)
    p[oracle.W1] = 1.0
    p[oracle.W2] = 1.0
    p[oracle.W3] = 1.0
    u = np.linspace(0.05, 0.95, 50)
    loss, g = oracle.mlp_loss_grad(p, u, u)
    assert loss < 1e-30 and np.abs(g).max() < 1e-15
    p[oracle.B3] = 0.125
    loss, g = oracle.mlp_loss_grad(p, u, u)
    assert abs(loss - 0.125**2) < 1e-15 and abs(g[oracle.B3] - 0.25) < 1e-15
    # dL/dW3[0] = mean(2 r h2) = 2 * 0.125 * mean(u)
    assert abs(g[oracle.W3] - 0.25 * u.mean()) < 1e-15


def test_tiny_network_closed_form():
    p = np.zeros(oracle.MLP_NP, dtype=np.float32)
    p[oracle.W1] = 2.0
    p[oracle.B1] = -0.5        # h1 = clamp(2u - 0.5)
    p[oracle.W2] = 1.0         # h2 = h1
    p[oracle.W3] = 0.5         # f = 0.5 h2 + 0.25
    p[oracle.B3] = 0.25
    for u, want in [(0.0, 0.25), (0.25, 0.25), (0.5, 0.5), (0.75, 0.75), (1.0, 0.75)]:
        assert oracle.mlp_forward(p, u) == want
    assert oracle.mlp_bucket(p, U64, 0, U64, 4096) == 3072


def _pieces(p):
    """ramps of an initialised map: (start u, end u, height) per used unit"""
    out = []
    for r in range(32):
        w, b, h = p[oracle.W1 + r], p[oracle.B1 + r], p[oracle.W3 + r]
        if h == 0:
            continue
        out.append((-b / w, (1 - b) / w, h))
    return out


@pytest.mark.parametrize("wl", ["gmm", "uniform", "dup_heavy"])
def test_init_interpolates_the_sample_cdf(wl):
    """f at the first and the last key of each piece equals the sample's CDF
    there (share of the sample before the piece, through the piece), up to
    the rounding of the heights to binary32, of W1/b1 and of the
    pre-activations; pieces tile the sample; the mixture's gaps are cut"""
    keys, _ = synth.make(wl, 50_000)
    s = np.sort(keys)
    smin, smax = int(s[0]), int(s[-1])
    p = oracle.mlp_init(s, smin, smax)
    m = s.size
    heights = p[oracle.W3:oracle.W3 + 32]
    assert abs(heights.sum() - 1.0) < 32 * 2.0**-24
    assert np.all(p[oracle.W1:oracle.W1 + 32] >= 0)
    cum = 0.0
    starts = []
    for lo, hi, h in _pieces(p):
        # lo, hi: the piece's first and last normalised key; f there
        f_lo = oracle.mlp_forward(p, lo)
        f_hi = oracle.mlp_forward(p, hi)
        tol = 64 * 2.0**-24
        assert abs(f_lo - cum) <= tol, (f_lo, cum)
        cum += h
        if hi > lo:
            assert abs(f_hi - cum) <= tol, (f_hi, cum)
        starts.append(lo)
    assert abs(cum - 1.0) < 32 * 2.0**-24
    assert starts == sorted(starts)
    if wl == "gmm":  # four separated components: the three gaps are cut
        assert len(_pieces(p)) >= 28 + 3


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_monotone_for_nonnegative_weights(seed):
    p = random_params(seed)
    us = np.linspace(0, 1, 20001)
    f = np.array([oracle.mlp_forward(p, float(u)) for u in us])
    assert np.all(np.diff(f) >= 0)


def test_thresholds_are_the_first_keys_of_each_bucket():
    p = random_params(7, scale=1.0)
    smin, smax = 10**15, 2**63 + 12345
    B = 64
    nt, t = oracle.mlp_thresholds(p, smin, smax, B)
    assert nt == oracle.mlp_bucket(p, U64, smin, smax, B)
    assert np.all(np.diff(t[:nt].astype(object)) >= 0)
    for b in range(1, nt + 1):
        x = int(t[b - 1])
        assert oracle.mlp_bucket(p, x, smin, smax, B) >= b
        if x > 0:
            assert oracle.mlp_bucket(p, x - 1, smin, smax, B) < b
    # bucket(x) == #{b : t_b <= x} on random keys
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2**64, size=300, dtype=np.uint64, endpoint=False):
        direct = oracle.mlp_bucket(p, int(x), smin, smax, B)
        via = int(np.count_nonzero(t[:nt] <= x))
        assert direct == via


def test_mid_rank_targets():
    s = np.array([5, 7, 7, 7, 9], dtype=np.uint64)
    y = oracle.mlp_targets(s)
    # (#{< x} + #{<= x}) / (2m): the middle of each key's run of ranks
    assert y.tolist() == [0.1, 0.5, 0.5, 0.5, 0.9]


def test_adam_first_step_is_lr_times_sign_and_keeps_weights_nonnegative():
    """Adam's first bias-corrected step is lr * g / (|g| + eps), i.e. lr * sign(g)
    for |g| >> eps; projected weights never go negative."""
    rng = np.random.default_rng(11)
    p = random_params(4)
    p[oracle.W3:oracle.W3 + 4] = 0.0          # on the boundary of the projection
    u = rng.uniform(0, 1, 64)
    y = np.sort(rng.uniform(0, 1, 64))
    _, g = oracle.mlp_loss_grad(p, u, y)
    lr = 2.0**-12
    p1, lf, ll = oracle.mlp_train(p, u, y, steps=1, batches=1, lr=lr)
    assert lf == ll
    big = np.abs(g) > 1e-6
    want = p.astype(np.float64) - lr * np.sign(g)
    wmask = np.zeros(oracle.MLP_NP, dtype=bool)
    wmask[oracle.W1:oracle.B1] = wmask[oracle.W2:oracle.B2] = wmask[oracle.W3:oracle.B3] = True
    want[wmask] = np.maximum(want[wmask], 0.0)
    tol = np.abs(want) * 2.0**-23 + lr * 1e-2
    assert np.all(np.abs(p1[big] - want[big]) <= tol[big])
    assert np.all(p1[wmask] >= 0)


def test_training_reduces_the_loss_on_a_mixture_sample():
    keys, _ = synth.make("gmm", 100_000)
    s = np.sort(keys[::50])
    smin, smax = int(s[0]), int(s[-1])
    p = oracle.mlp_init(s, smin, smax)
    u = np.array([oracle.mlp_norm(int(x), smin, smax) for x in s])
    y = oracle.mlp_targets(s)
    l0, _ = oracle.mlp_loss_grad(p, u, y)
    p2, _, _ = oracle.mlp_train(p, u, y, steps=48, batches=8, lr=1e-3)
    l1, _ = oracle.mlp_loss_grad(p2, u, y)
    assert l1 < 0.8 * l0
    # still monotone after training (projection)
    f = np.array([oracle.mlp_forward(p2, float(v)) for v in np.linspace(0, 1, 5001)])
    assert np.all(np.diff(f) >= 0)


# ---------------------------------------------------------------------------
# Adam over several steps: a hand-derived golden (tests/golden/adam_three_steps.json)
# ---------------------------------------------------------------------------
import json
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adam_three_steps.json")


def _f32_ulp(v):
    v = np.float32(v)
    return float(np.spacing(np.abs(v))) if v != 0 else float(np.spacing(np.float32(0)))


def _adam_case(case):
    p = np.zeros(oracle.MLP_NP, dtype=np.float64)
    free = [oracle.B3]
    if "W3_0_init" in case:
        p[oracle.W3] = case["W3_0_init"]
        p[oracle.B2] = 1.0
        free.append(oracle.W3)
    u = np.array([0.1, 0.2, 0.3, 0.4])
    y = np.array(case["targets"], dtype=np.float64)
    return p, u, y, free


@pytest.mark.parametrize("name", ["case_A", "case_B"])
def test_adam_three_steps_match_hand_derivation(name):
    """Parameters after 1, 2 and 3 Adam steps equal the values worked out by
    hand from the published algorithm (running powers of beta1/beta2, bias
    correction of each moment, minibatch t mod nb, binary32 rounding and the
    projection of weights, with the moments kept across a projection)."""
    g = json.load(open(GOLDEN))
    case = g[name]
    p0, u, y, free = _adam_case(case)
    for st in case["steps"]:
        t = st["t"]
        p, lf, ll = oracle.mlp_train(p0, u, y, steps=t, batches=case["batches"], lr=g["lr"])
        want = {oracle.B3: st["b3"]}
        if "W3_0" in st:
            want[oracle.W3] = st["W3_0"]
        for idx, v in want.items():
            # binary32 parameters: the hand value rounded to binary32 (one ulp
            # of slack for the last bit of the unrounded step)
            assert abs(p[idx] - v) <= _f32_ulp(v), (name, t, idx, p[idx], v)
        # every parameter without a gradient is untouched
        other = np.ones(oracle.MLP_NP, dtype=bool)
        other[free] = False
        assert np.array_equal(p[other], oracle._par(p0)[other]), (name, t)
        assert abs(lf - case["steps"][0]["loss_before"]) <= 1e-12 * case["steps"][0]["loss_before"]
        assert abs(ll - st["loss_before"]) <= 1e-9 * st["loss_before"] + 1e-15, (name, t, ll)
    if name == "case_B":
        # projected to exactly 0 after step 1, positive again after step 2
        p1, _, _ = oracle.mlp_train(p0, u, y, steps=1, batches=1, lr=g["lr"])
        assert p1[oracle.W3] == 0.0 and p1[oracle.B3] < 0.0


# ---------------------------------------------------------------------------
# key normalisation u(x) = (x - smin) / (smax - smin) inside the range
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("smin,smax,x,want", [
    (0, 2**40, 2**39, 0.5),
    (0, 2**40, 2**38, 0.25),
    (0, 2**40, 3 * 2**38, 0.75),
    (2**20, 2**20 + 2**40, 2**20 + 2**39, 0.5),
    (10, 110, 35, 0.25),
    (10, 110, 60, 0.5),
    (10, 110, 11, 0.01),
    (2**63, 2**64 - 1, 2**63 + 2**62, 0.5),
    (5, 7, 6, 0.5),
])
def test_norm_interior_closed_forms(smin, smax, x, want):
    """Inside (smin, smax) the normalised key is the exact ratio of the key's
    offset from smin to the range, correctly rounded; the ends clamp."""
    assert oracle.mlp_norm(x, smin, smax) == want
    assert oracle.mlp_norm(smin, smin, smax) == 0.0
    assert oracle.mlp_norm(smax, smin, smax) == 1.0
    assert oracle.mlp_norm(max(smin, 1) - 1, smin, smax) == 0.0
