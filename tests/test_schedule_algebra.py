"""Host-side check of the algebra behind the conjugate-symmetric batched schedule.

A plain Python model of the schedule's passes (the step order of a row, the
symmetrised weights of each unordered pair, pass A on the plane-zeroed copy of
fhat, the edge passes E1/E2/E3 on axis-permuted copies, pass Z, and the final
assembly) is compared with the direct sum of Sec. 3.2 for an fhat that is the
transform of a real f on the asymmetric mesh.  The weight is an arbitrary
function of the integer norms (n_a, n_b, n_c), the only property the schedule
relies on.  The GPU tests check the library itself against the oracle.
"""
import numpy as np
import pytest


def _model(N, seed=0, core_r2=-1):
    """With core_r2 >= 0 the pairs whose two partners lie in the ball |m - N/2|^2 <= core_r2
    get weight 0 in every pass and are summed separately over every output (the
    FP64 core of the batched FP32 mode), then added after the assembly."""
    h = N // 2
    rng = np.random.default_rng(seed)
    lo = lambda k: max(0, k - h + 1)
    hi = lambda k: min(N - 1, k + h)
    cnt = lambda k: hi(k) - lo(k) + 1

    def steps_of(k1, k2):
        out = []
        for m1 in range(lo(k1), min((k1 + h) // 2, hi(k1)) + 1):
            last = hi(k2) if 2 * m1 < k1 + h else min((k2 + h) // 2, hi(k2))
            out += [(m1, m2) for m2 in range(lo(k2), last + 1)]
        return out

    Tg = rng.standard_normal((3 * N * N, 3 * N * N))   # "gain" part, indexed (n_a, n_b)
    Tl = rng.standard_normal(3 * N * N)                # "loss" part, indexed n_c

    def sq(v):
        return sum(x * x for x in v)

    def w_ordered(k, m):
        return Tg[sq([a - h for a in k]), sq([2 * b - a - h for a, b in zip(k, m)])] - Tl[sq([b - h for b in m])]

    def w_pair(k, m, j, core=False):
        na, nb = sq([a - h for a in k]), sq([a - b for a, b in zip(m, j)])
        ncm, ncj = sq([a - h for a in m]), sq([a - h for a in j])
        if (ncm <= core_r2 and ncj <= core_r2) != core:
            return 0.0
        if (m[0], m[1]) == (j[0], j[1]):
            if m[2] == j[2]:
                return Tg[na, 0] - Tl[ncm]
            if m[2] > j[2]:
                return 0.0
        return 2 * Tg[na, nb] - Tl[ncm] - Tl[ncj]

    f = rng.standard_normal((N, N, N))
    v = np.arange(N) - h
    E = np.exp(-2j * np.pi / N * np.outer(v, v))
    fh = np.einsum("ai,bj,ck,ijk->abc", E, E, E, f)

    def run_row(F, a, b, s0, s1, zero_inner_edges=False):
        out = np.zeros(N, complex)
        for (m1, m2) in steps_of(a, b)[s0:s1]:
            j1, j2 = a + h - m1, b + h - m2
            for k3 in range(N):
                for m3 in range(lo(k3), hi(k3) + 1):
                    j3 = k3 + h - m3
                    w = w_pair((a, b, k3), (m1, m2, m3), (j1, j2, j3))
                    if zero_inner_edges and k3 < h and (m3 == 0 or m3 == k3 + h):
                        w = 0.0
                    out[k3] += w * F[m1, m2, m3] * F[j1, j2, j3]
        return out

    derived = lambda k1, k2: k1 >= 1 and k2 >= 1 and (k1 > h or (k1 == h and k2 > h))
    g = fh.copy()
    g[0], g[:, 0], g[:, :, 0] = 0, 0, 0
    F213, F312 = fh.transpose(1, 0, 2), fh.transpose(2, 0, 1)
    A, E1, E2, E3, Z = (np.zeros((N, N, N), complex) for _ in range(5))
    for k1 in range(N):
        for k2 in range(N):
            if not derived(k1, k2):
                A[k1, k2] = run_row(g, k1, k2, cnt(k2) if k1 < h else 0, len(steps_of(k1, k2)))
    for a in range(h):
        for b in range(N):
            c, cut = cnt(b), (1 if b < h else 0)
            E1[a, b] = run_row(fh, a, b, 0, c)
            E2[a, b] = run_row(F213, a, b, cut, c - cut)
            E3[a, b] = run_row(F312, a, b, cut, c - cut, zero_inner_edges=True)
    for b in range(h, N):
        Z[0, b] = run_row(F312, 0, b, 0, len(steps_of(0, b)))

    def edge(x1, x2, x3):
        return ((E1[x1, x2, x3] if x1 < h else 0) + (E2[x2, x1, x3] if x2 < h else 0)
                + (E3[x3, x1, x2] if x3 < h else 0))

    # core: every output, unordered pairs of core rows (m1, m2) <= (j1, j2), m3 <= j3 on the diagonal
    C = np.zeros((N, N, N), complex)
    if core_r2 >= 0:
        r = int(np.floor(np.sqrt(core_r2)))
        disk = [(a, b) for a in range(N) for b in range(N) if (a - h) ** 2 + (b - h) ** 2 <= core_r2]
        for k1 in range(N):
            for k2 in range(N):
                for (m1, m2) in disk:
                    j1, j2 = k1 + h - m1, k2 + h - m2
                    if (j1, j2) not in disk or (m1, m2) > (j1, j2):
                        continue
                    for m3 in range(h - r, h + r + 1):
                        for j3 in range(h - r, h + r + 1):
                            k3 = m3 + j3 - h
                            if 0 <= k3 < N:
                                w = w_pair((k1, k2, k3), (m1, m2, m3), (j1, j2, j3), core=True)
                                C[k1, k2, k3] += w * fh[m1, m2, m3] * fh[j1, j2, j3]
    got = np.zeros((N, N, N), complex)
    want = np.zeros((N, N, N), complex)
    for k1 in range(N):
        for k2 in range(N):
            for k3 in range(N):
                if not derived(k1, k2):
                    got[k1, k2, k3] = A[k1, k2, k3] + edge(k1, k2, k3)
                elif k3 == 0:
                    got[k1, k2, k3] = Z[0, k1, k2]
                else:
                    got[k1, k2, k3] = np.conj(A[N - k1, N - k2, N - k3]) + edge(k1, k2, k3)
                # the core is summed for the direct rows (and k3 = 0 of the derived rows);
                # a derived output with k3 >= 1 takes the conjugate of its mirror's
                if derived(k1, k2) and k3 >= 1:
                    got[k1, k2, k3] += np.conj(C[N - k1, N - k2, N - k3])
                else:
                    got[k1, k2, k3] += C[k1, k2, k3]
                k = (k1, k2, k3)
                for m1 in range(lo(k1), hi(k1) + 1):
                    for m2 in range(lo(k2), hi(k2) + 1):
                        for m3 in range(lo(k3), hi(k3) + 1):
                            j = (k1 - m1 + h, k2 - m2 + h, k3 - m3 + h)
                            want[k] += w_ordered(k, (m1, m2, m3)) * fh[m1, m2, m3] * fh[j]
    return got, want


@pytest.mark.parametrize("N", [8])
def test_conjugate_symmetric_schedule_reproduces_the_direct_sum(N):
    got, want = _model(N)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("core_r2", [0, 2, 5, 9])
def test_core_split_reproduces_the_direct_sum(core_r2):
    """The FP32 passes without the core-core pairs, plus the core sum of the direct rows
    (and of k3 = 0 of the derived rows) with the derived outputs taken as conjugates of their
    mirrors, equal the direct sum; r2 = 9 at N = 8 (r = 3) makes core outputs reach k_d = 0."""
    got, want = _model(8, seed=2, core_r2=core_r2)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_planted_mistake_is_caught():
    """Dropping the edge correction of the mirrored outputs must fail the comparison."""
    N, h = 8, 4
    got, want = _model(N, seed=1)
    # the mirrored outputs with k3 >= 1 carry E(k); an assembly without it differs there
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    derived = [(a, b) for a in range(N) for b in range(N) if a >= 1 and b >= 1 and (a > h or (a == h and b > h))]
    bad = got.copy()
    for a, b in derived:
        bad[a, b, 1:] = np.conj(got[N - a, N - b, N - 1:0:-1])
    assert np.max(np.abs(bad - want)) > 1e-6 * np.max(np.abs(want))
