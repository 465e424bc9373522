"""Pins for the oracle's integer and double X-engine (no GPU).

The product is V_ij = sum_t x_i(t) conj(x_j(t)) per channel (the FX correlator's
cross-multiply; paper Sec. 2.2 linear algebra, Sec. 7 correlation).  The oracle is
checked against hand-expanded sums, brute force in Python complex integers,
numpy's einsum, closed forms and invariants, so that a dropped term, a wrong sign,
a swapped (i, j) or a wrong packing index each fails at least one test.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from conftest import GOLDEN


def _read_nibbles():
    tab = {}
    with open(os.path.join(GOLDEN, "ci4_nibble_table.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                n, v = line.split()
                tab[int(n)] = int(v)
    assert len(tab) == 16
    return tab


def _read_hand_cases():
    cases = []
    with open(os.path.join(GOLDEN, "xengine_hand.txt")) as fh:
        lines = [l.split("#")[0].strip() for l in fh]
    lines = [l for l in lines if l]
    k = 0
    while k < len(lines):
        head = lines[k].split()
        assert head[0] == "case"
        name, dtype = head[1], head[2]
        T, F, N = map(int, head[3:6])
        k += 1
        re = np.zeros((T, F, N), np.int64)
        im = np.zeros((T, F, N), np.int64)
        for _ in range(T * F * N):
            t, f, i, r, m = map(int, lines[k].split())
            re[t, f, i], im[t, f, i] = r, m
            k += 1
        expect = {}
        while lines[k] != "end":
            f, p, r, m = map(int, lines[k].split())
            expect[(f, p)] = (r, m)
            k += 1
        k += 1
        cases.append((name, dtype, T, F, N, re, im, expect))
    return cases


def _pack(dtype, re, im):
    return synth.pack_ci4(re, im) if dtype == "ci4" else synth.pack_ci8(re, im)


# ---------------------------------------------------------------- unpack

def test_unpack_ci4_exhaustive_against_hand_table():
    tab = _read_nibbles()
    b = np.arange(256, dtype=np.uint8)
    re, im = oracle.unpack_ci4(b)
    for v in range(256):
        assert re[v] == tab[v >> 4] and im[v] == tab[v & 15], v


def test_unpack_ci8_exhaustive():
    vals = np.arange(-128, 128)
    rr, ii = np.meshgrid(vals, vals, indexing="ij")
    pairs = synth.pack_ci8(rr, ii)
    re, im = oracle.unpack_ci8(pairs)
    assert np.array_equal(re, rr) and np.array_equal(im, ii)


def test_pack_ci4_roundtrip_all_values():
    vals = np.arange(-8, 8)
    rr, ii = np.meshgrid(vals, vals, indexing="ij")
    re, im = oracle.unpack_ci4(synth.pack_ci4(rr, ii))
    assert np.array_equal(re, rr) and np.array_equal(im, ii)
    # every byte value is reached exactly once
    assert len(set(synth.pack_ci4(rr, ii).ravel().tolist())) == 256


# ---------------------------------------------------------------- X-engine

@pytest.mark.parametrize("case", _read_hand_cases(), ids=lambda c: c[0])
def test_xengine_hand_expanded(case):
    name, dtype, T, F, N, re, im, expect = case
    out = oracle.xengine_int(_pack(dtype, re, im), dtype, T, F, N)
    assert out.shape == (F, N * (N + 1) // 2, 2)
    for (f, p), (r, m) in expect.items():
        assert tuple(out[f, p]) == (r, m), (name, f, p)


def _brute(re, im):
    """Python complex-integer brute force, full matrix, [F][N][N] of (re, im)."""
    T, F, N = re.shape
    V = np.zeros((F, N, N, 2), np.int64)
    for f in range(F):
        for i in range(N):
            for j in range(N):
                sr = si = 0
                for t in range(T):
                    a = complex(int(re[t, f, i]), int(im[t, f, i]))
                    b = complex(int(re[t, f, j]), int(im[t, f, j]))
                    z = a * b.conjugate()
                    sr += int(z.real)
                    si += int(z.imag)
                V[f, i, j] = (sr, si)
    return V


def _tri(N):
    return [(i, j) for i in range(N) for j in range(i + 1)]


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
@pytest.mark.parametrize("T,F,N", [(1, 1, 1), (3, 2, 4), (2, 3, 3), (5, 1, 4)])
def test_xengine_brute_force_tiny(dtype, T, F, N):
    raw = synth.extreme_voltages(7 + T + F + N, T, F, N, dtype)
    re, im = (oracle.unpack_ci4(raw) if dtype == "ci4" else oracle.unpack_ci8(raw))
    V = _brute(re, im)
    out = oracle.xengine_int(raw, dtype, T, F, N)
    full = oracle.xengine_int(raw, dtype, T, F, N, full=True)
    assert np.array_equal(full, V)
    for p, (i, j) in enumerate(_tri(N)):
        assert np.array_equal(out[:, p], V[:, i, j])


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_xengine_matches_einsum(dtype):
    T, F, N = 37, 5, 24
    raw = synth.extreme_voltages(3, T, F, N, dtype)
    re, im = (oracle.unpack_ci4(raw) if dtype == "ci4" else oracle.unpack_ci8(raw))
    re = re.astype(np.int64)
    im = im.astype(np.int64)
    vr = np.einsum("tfi,tfj->fij", re, re) + np.einsum("tfi,tfj->fij", im, im)
    vi = np.einsum("tfi,tfj->fij", im, re) - np.einsum("tfi,tfj->fij", re, im)
    full = oracle.xengine_int(raw, dtype, T, F, N, full=True)
    assert np.array_equal(full[..., 0], vr)
    assert np.array_equal(full[..., 1], vi)


def test_xengine_invariants():
    T, F, N = 50, 3, 16
    raw = synth.voltages(11, T, F, N, "ci8", 8.0, 127)
    full = oracle.xengine_int(raw, "ci8", T, F, N, full=True)
    # Hermitian: V_ji = conj(V_ij)
    assert np.array_equal(full[..., 0], np.swapaxes(full[..., 0], 1, 2))
    assert np.array_equal(full[..., 1], -np.swapaxes(full[..., 1], 1, 2))
    # autocorrelations are real and non-negative
    d = np.arange(N)
    assert np.all(full[:, d, d, 1] == 0)
    assert np.all(full[:, d, d, 0] >= 0)
    # Cauchy-Schwarz |V_ij|^2 <= V_ii V_jj
    mag2 = full[..., 0].astype(float) ** 2 + full[..., 1].astype(float) ** 2
    aa = full[:, d, d, 0].astype(float)
    assert np.all(mag2 <= aa[:, :, None] * aa[:, None, :] + 1e-6)


def test_xengine_linear_in_time():
    T, F, N = 40, 2, 12
    raw = synth.voltages(12, T, F, N, "ci4", 2.5, 7)
    whole = oracle.xengine_int(raw, "ci4", T, F, N)
    a = oracle.xengine_int(raw, "ci4", T, F, N, t0=0, nt=17)
    b = oracle.xengine_int(raw, "ci4", T, F, N, t0=17, nt=T - 17)
    assert np.array_equal(whole, a + b)
    # channel subsets agree with the whole
    sub = oracle.xengine_int(raw, "ci4", T, F, N, chans=(1, 1))
    assert np.array_equal(sub[0], whole[1])


def test_xengine_permutation_equivariant():
    T, F, N = 20, 2, 10
    raw = synth.voltages(13, T, F, N, "ci8", 8.0, 127)
    perm = np.random.default_rng(0).permutation(N)
    full = oracle.xengine_int(raw, "ci8", T, F, N, full=True)
    fullp = oracle.xengine_int(np.ascontiguousarray(raw[:, :, perm]), "ci8", T, F, N, full=True)
    assert np.array_equal(fullp, full[:, perm][:, :, perm])


@pytest.mark.parametrize("c", [(3, -2), (-8, 7), (0, -8)])
def test_xengine_constant_input_closed_form(c):
    # x_t = c for every input and sample: V_ij = T |c|^2, Im = 0
    T, F, N = 9, 2, 5
    raw = synth.constant_voltages(T, F, N, "ci4", *c)
    out = oracle.xengine_int(raw, "ci4", T, F, N)
    assert np.all(out[..., 0] == T * (c[0] ** 2 + c[1] ** 2))
    assert np.all(out[..., 1] == 0)


def test_xengine_single_sample_outer_product():
    # one nonzero sample gives the outer product x x^H
    T, F, N = 4, 1, 6
    re = np.zeros((T, F, N), int)
    im = np.zeros((T, F, N), int)
    rng = np.random.default_rng(5)
    re[2, 0] = rng.integers(-8, 8, N)
    im[2, 0] = rng.integers(-8, 8, N)
    out = oracle.xengine_int(synth.pack_ci4(re, im), "ci4", T, F, N)
    z = re[2, 0] + 1j * im[2, 0]
    for p, (i, j) in enumerate(_tri(N)):
        v = z[i] * np.conj(z[j])
        assert out[0, p, 0] == int(v.real) and out[0, p, 1] == int(v.imag)


def test_xengine_rotating_phasor_closed_form():
    # x_i(t) = (a_i + i b_i) * i^t: every sample has the same conjugate
    # product, so V_ij = T (a_i + i b_i)(a_j - i b_j) exactly.
    T, F, N = 12, 1, 4
    rng = np.random.default_rng(9)
    z0 = rng.integers(-7, 8, N) + 1j * rng.integers(-7, 8, N)
    zt = np.array([z0 * (1j ** t) for t in range(T)])
    re = np.rint(zt.real).astype(int)[:, None, :]
    im = np.rint(zt.imag).astype(int)[:, None, :]
    out = oracle.xengine_int(synth.pack_ci8(re, im), "ci8", T, F, N)
    for p, (i, j) in enumerate(_tri(N)):
        v = T * z0[i] * np.conj(z0[j])
        assert out[0, p, 0] == int(v.real) and out[0, p, 1] == int(v.imag)


def test_xengine_autocorrelation_statistics():
    # E[V_ii] = T E|x|^2 for rounded Gaussians sigma=8 clipped at 127
    T, F, N = 512, 8, 32
    raw = synth.voltages(1, T, F, N, "ci8", 8.0, 127)
    out = oracle.xengine_int(raw, "ci8", T, F, N)
    auto = np.array([out[:, i * (i + 1) // 2 + i, 0] for i in range(N)], float)
    # E|x|^2 = 2 E[rint(8z)^2] = 2 (64 + 1/12) (Sheppard), per-sample var ~ 2*2*64^2
    expect = T * 2 * (64 + 1.0 / 12)
    se = np.sqrt(T * 4 * 64.0 ** 2) / np.sqrt(auto.size)
    assert abs(auto.mean() - expect) < 5 * se


def test_xengine_freivalds_identity_on_oracle():
    # V r = sum_t x_t (x_t^H r) exactly, for the Hermitian V rebuilt from the
    # lower triangle.  The same check is used on large GPU outputs.
    from fx_checks import freivalds_check
    T, F, N = 30, 3, 20
    raw = synth.voltages(21, T, F, N, "ci8", 8.0, 127)
    out = oracle.xengine_int(raw, "ci8", T, F, N)
    re, im = oracle.unpack_ci8(raw)
    assert freivalds_check(out, re, im, seed=1)
    bad = out.copy()
    bad[1, 7, 1] += 1
    assert not freivalds_check(bad, re, im, seed=1)
    # large vectors push the a priori bound past 2^53: the int64 path
    big = synth.extreme_voltages(22, 512, 2, 32, "ci8")
    vb = oracle.xengine_int(big, "ci8", 512, 2, 32)
    bre, bim = oracle.unpack_ci8(big)
    assert freivalds_check(vb, bre, bim, seed=2, rmax=1 << 24)
    vb[1, 100, 0] -= 1
    assert not freivalds_check(vb, bre, bim, seed=2, rmax=1 << 24)


def test_xengine_f64_matches_int_on_integer_data():
    T, F, N = 16, 2, 9
    raw = synth.voltages(4, T, F, N, "ci8", 8.0, 127)
    re, im = oracle.unpack_ci8(raw)
    a = oracle.xengine_int(raw, "ci8", T, F, N)
    b = oracle.xengine_f64(re, im)
    assert np.array_equal(a.astype(np.float64), b)


def test_xengine_f64_half_values_exact():
    # FP16 inputs: products are exact in double; a sum of few terms is exact too
    T, F, N = 3, 1, 2
    x = np.array([[[[0.5, -1.25], [2.0, 0.125]]], [[[1.0, 0.0], [-0.5, 0.5]]],
                  [[[0.0, 3.0], [1.5, -2.0]]]])
    re, im = x[..., 0], x[..., 1]
    out = oracle.xengine_f64(re, im)
    z = re + 1j * im
    v10 = np.sum(z[:, 0, 1] * np.conj(z[:, 0, 0]))
    assert out[0, 1, 0] == v10.real and out[0, 1, 1] == v10.imag


def test_accumulate_f64_k_identical_dumps():
    d = np.random.default_rng(2).standard_normal(1000).astype(np.float32).astype(np.float64)
    run = np.zeros_like(d)
    for _ in range(8):
        oracle.accumulate_f64(run, d)
    assert np.array_equal(run, 8 * d)
