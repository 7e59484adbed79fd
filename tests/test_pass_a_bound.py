"""The first distance pass's flag bound against a model of its arithmetic (CPU).

The first pass (split-FP16 matrix-core variant) scores a pair (p, o) of a query block
with centre c as
    t_A = |p'|^2 + [n_hi + n_lo - 2 (o_hi.p_hi + o_lo.p_hi + o_hi.p_lo + o_lo.p_lo)]
where p' = fl32(p - c), o' = fl32(o - c), every coordinate v is split as hi = f16(v),
lo = f16(fl32(v - hi)), n = fl32(|o'|^2), the 16 half-precision products are exact and
are summed in single precision in an order the hardware does not document.  The block's
flag bound is thr = d_max^2 + 2^-15 (R + d_max)^2 + 1e-6 (R: the block radius about c);
the exact pass relies on t_A < thr for every pair with |p - o| < d_max (Sec. IV-C: the
collision penalty is zero from d_max on, so only those pairs may decide a cost).

Derivation of the error of t_A for a pair with |p - o| <= d_max, S = (R + d_max)^2,
u = 2^-24 (so |p'| <= R and |o'| <= R + d_max):
  * recentring: |(p' - o') - (p - o)| <= 2 sqrt(3) u (R + d_max) per pair, changing
    |p' - o'|^2 by at most ~7 u d_max (2 R + d_max) <= 14 u S;
  * |p'|^2 and n in single precision (one multiply, two FMAs): <= 3 u S each;
  * split: |v - (hi + lo)| <= 2^-22 |v| (lo rounds a residual of at most 2^-11 |v| to
    11 bits), or <= 2^-25 absolute when lo is subnormal in half precision; the cross
    terms (o_hi + o_lo).(p_hi + p_lo) then differ from -2 o'.p' by <= 2^-20 |o'||p'|
    <= 16 u S, the norm by <= 2^-22 S = 4 u S (absolute subnormal parts: <= 2^-22
    (R + d_max), inside the 1e-6 term while R + d_max <= 4 m and inside the relative
    term beyond);
  * accumulation: 16 exact products summed with at most 15 single-precision roundings
    in any order: <= 15 u sum |a_k b_k| <= 15 u (|o'|^2 + 2 |o'||p'|) <= 45 u S (wider
    internal precision or fewer roundings only lower this);
  * the final single-precision add: <= u S.
Total <= 14 + 6 + 16 + 4 + 45 + 1 = 86 u S ~ 2^-17.6 S, a factor of 6 under the
2^-15 S of the bound.  The tests below evaluate t_A in this model on inputs chosen to
make each term large (coordinates on half-precision rounding boundaries, blocks at
the largest radius the variant accepts, pairs at d_max) and check the bound, and that
the check is not vacuous: the worst error found is above 2^-23 S (about 2^-21 S on these
inputs, some 70 times under the bound), and the model with one cross term dropped
breaks the bound.
"""
import itertools

import numpy as np

F32, F16 = np.float32, np.float16
U = 2.0 ** -24


def f32(x):
    return np.asarray(x, np.float64).astype(F32)


def split(v):
    """hi = f16(v), lo = f16(fl32(v - hi)), as float64 values."""
    v = f32(v)
    hi = v.astype(F16)
    lo = (v - hi.astype(F32)).astype(F32).astype(F16)
    return hi.astype(np.float64), lo.astype(np.float64)


def fma32(a, b, c):
    """Single-precision fused multiply-add (one rounding): exact in float64 for
    float32 operands' product plus a float32 addend, then rounded once."""
    return f32(np.float64(a) * np.float64(b) + np.float64(c))


def norm32(x, y, z):
    return fma32(z, z, fma32(y, y, f32(np.float64(x) * np.float64(x))))


def sum32(terms, order):
    """Products summed in single precision in the given order (each add rounds)."""
    acc = F32(0.0)
    for k in order:
        acc = f32(np.float64(acc) + terms[k])
    return acc


ORDERS = [list(range(16)), list(range(15, -1, -1))]


def pass_a_value(p, o, c, orders=ORDERS):
    """Model of t_A for one pair in the given summation orders (list of values)."""
    pp_ = [f32(np.float64(f32(p[a])) - np.float64(f32(c[a]))) for a in range(3)]
    oo_ = [f32(np.float64(f32(o[a])) - np.float64(f32(c[a]))) for a in range(3)]
    pp = norm32(*pp_)
    n = norm32(*oo_)
    m2o = [f32(-2.0 * np.float64(v)) for v in oo_]
    ah = [split(v) for v in m2o]            # -2 o' halves
    nh = split(n)
    ph = [split(v) for v in pp_]            # p' halves
    # K = 16 slots: [-2o_hi, n_hi, -2o_lo, n_lo | -2o_hi, n_hi, -2o_lo, n_lo]
    #            x  [  p_hi,    1,   p_hi,    1 |   p_lo,    0,   p_lo,    0]
    terms = []
    for a in range(3):
        terms.append(ah[a][0] * ph[a][0])
    terms.append(nh[0])
    for a in range(3):
        terms.append(ah[a][1] * ph[a][0])
    terms.append(nh[1])
    for a in range(3):
        terms.append(ah[a][0] * ph[a][1])
    terms.append(0.0)
    for a in range(3):
        terms.append(ah[a][1] * ph[a][1])
    terms.append(0.0)
    out = []
    for order in orders:
        t = sum32(terms, order)
        out.append(float(f32(np.float64(pp) + np.float64(t))))
    return out


def flag_bound(R, d_max):
    span = R * 1.001 + d_max
    return d_max * d_max + 2.0 ** -15 * span * span + 1e-6


def adversarial_pairs(rng, R, d_max, n):
    """Blocks of radius R about a centre far from the origin (large coordinates make the
    recentring round), queries on the block's sphere, points at distance just under
    d_max from them, with coordinates nudged onto half-precision rounding boundaries."""
    out = []
    while len(out) < n:
        c = rng.uniform(-40.0, 40.0, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        p = c + R * d
        # the point continues outward (|o'| = R + d_max: the largest cross terms)
        e = d + 0.05 * rng.normal(size=3)
        e /= np.linalg.norm(e)
        o = p + d_max * (1.0 - 1e-7) * e
        # nudge a recentred coordinate onto a half-precision tie (largest lo)
        a = rng.integers(3)
        v = F32(o[a] - c[a])
        hi = np.float64(F16(v))
        ulp = np.spacing(F16(abs(hi) if hi != 0 else 1.0)).astype(np.float64)
        o[a] = c[a] + hi + 0.5 * ulp * np.sign(v if v != 0 else 1.0) * (1.0 - 2.0 ** -12)
        p32, o32 = f32(p), f32(o)
        # keep the pairs the nudge left within d_max (about half): they lie at the bound
        if np.sum((p32.astype(np.float64) - o32.astype(np.float64)) ** 2) < d_max * d_max:
            out.append((p32, o32, f32(c)))
    return out


def test_split_f16_bound_holds_on_adversarial_pairs():
    rng = np.random.default_rng(11)
    worst_ratio = 0.0
    rand_orders = ORDERS + [list(rng.permutation(16)) for _ in range(6)]
    for R, d_max in [(0.5, 1.0), (4.0, 1.0), (20.0, 1.0), (63.0 - 1.0, 1.0),
                     (30.0, 3.0), (2.0, 0.2)]:
        thr = flag_bound(R, d_max)
        S = (R + d_max) ** 2
        for p, o, c in adversarial_pairs(rng, R, d_max, 150):
            exact = float(np.sum((p.astype(np.float64) - o.astype(np.float64)) ** 2))
            assert exact < d_max * d_max
            for tA in pass_a_value(p, o, c, rand_orders):
                assert tA < thr, (R, d_max, tA, thr)
                worst_ratio = max(worst_ratio, abs(tA - exact) / S)
    # the inputs do reach the rounding terms (not a vacuous check) and stay well
    # inside 2^-15 (the derivation allows up to ~2^-17.6)
    assert worst_ratio > 2.0 ** -23
    assert worst_ratio < 2.0 ** -15


def test_model_catches_a_dropped_cross_term():
    """The same model with the o_lo.p_hi products dropped (a plausible slot-layout
    mistake) breaks the bound on these inputs: the check can fail."""
    rng = np.random.default_rng(12)
    R, d_max = 40.0, 1.0
    thr = flag_bound(R, d_max)
    broke = False
    for p, o, c in adversarial_pairs(rng, R, d_max, 60):
        pp_ = [f32(np.float64(p[a]) - np.float64(c[a])) for a in range(3)]
        oo_ = [f32(np.float64(o[a]) - np.float64(c[a])) for a in range(3)]
        n = norm32(*oo_)
        hi_lo = [split(f32(-2.0 * np.float64(v))) for v in oo_]
        ph = [split(v) for v in pp_]
        t = sum(hi_lo[a][0] * ph[a][0] + hi_lo[a][0] * ph[a][1] + hi_lo[a][1] * ph[a][1]
                for a in range(3)) + sum(split(n))
        tA = float(norm32(*pp_)) + t
        exact = float(np.sum((p.astype(np.float64) - o.astype(np.float64)) ** 2))
        if abs(tA - exact) > thr - d_max * d_max:
            broke = True
            break
    assert broke


def test_far_points_cannot_be_within_reach():
    """Points with |o'| >= 128 get t = 32768 in the pass; with R + d_max <= 64 (the
    variant's condition for a finite bound) such a point is farther than 64 - R >=
    d_max from every query of the block, so no pair within d_max is lost."""
    for R, d_max in itertools.product([0.0, 10.0, 63.0], [0.5, 1.0]):
        if R + d_max > 64.0:
            continue
        assert 128.0 - R > d_max
        assert 32768.0 >= flag_bound(R, d_max)
