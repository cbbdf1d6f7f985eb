"""CPU model of the out-of-core schedule of eor_loglike_host (host loop of
csrc/ooc.hip): the same packing of tile columns, pass width, window sizes
and workgroup-to-tile mappings (window and within-pass updates), on small
tiles in numpy. It checks that every
index stays inside the buffers the library allocates and that the schedule
computes the Cholesky factor (against numpy), for windows from the smallest
allowed to roomy ones and for ragged tile counts."""
import numpy as np
import pytest


def _schedule(n, avail, bs=4, seed=0):
    rng = np.random.default_rng(seed)
    N = (n + bs - 1) // bs
    npad = N * bs
    M = rng.standard_normal((npad, npad)) + 1j * rng.standard_normal((npad, npad))
    S = M @ M.conj().T + npad * np.eye(npad)
    col_off = lambda k: k * N - k * (k - 1) // 2
    ntile = N * (N + 1) // 2
    Ah = [None] * ntile
    for k in range(N):
        for i in range(k, N):
            Ah[col_off(k) + i - k] = S[i * bs:(i + 1) * bs, k * bs:(k + 1) * bs].copy()
    Lh = [None] * ntile      # the host factor: only what later passes read is written back
    done = [None] * ntile    # every finished tile, to check the factor
    cols = avail // N                      # full-height tile columns that fit (>= 2)
    J = min(N, cols - min(4, cols // 2))   # the window keeps min(4, half) of them
    capC, cap = J * N, avail - J * N
    assert cap >= N
    for j0 in range(0, N, J):
        j1 = min(N, j0 + J)
        nt, rows0 = col_off(j1) - col_off(j0), N - j0
        assert nt <= capC
        C = [Ah[col_off(j0) + t].copy() for t in range(nt)]
        W = max(1, min(j0, cap // rows0))
        for k0 in range(0, j0, W):
            wk = min(W, j0 - k0)
            assert wk * rows0 <= cap
            Lw = [None] * (wk * rows0)
            for k in range(wk):
                kk = k0 + k
                for r in range(rows0):
                    src = col_off(kk) + (j0 - kk) + r
                    assert col_off(kk) <= src < col_off(kk + 1)
                    assert Lh[src] is not None, "a window reads a tile that was never written back"
                    Lw[k * rows0 + r] = Lh[src]
            for blk in range(nt):  # workgroup -> tile (i, j) as ooc_window_kernel maps it
                b, j = blk, j0
                while j < j1 - 1 and b >= N - j:
                    b -= N - j
                    j += 1
                i = j + b
                assert i < N
                C[blk] = C[blk] - sum(Lw[k * rows0 + (i - j0)] @ Lw[k * rows0 + (j - j0)].conj().T
                                      for k in range(wk))
        loc = lambda k: (k - j0) * N - ((k * (k - 1)) // 2 - (j0 * (j0 - 1)) // 2)
        for j in range(j0, j1):
            assert loc(j) == col_off(j) - col_off(j0)
            Ljj = np.linalg.cholesky(C[loc(j)])
            C[loc(j)] = Ljj
            Linv = np.linalg.inv(Ljj)
            for t in range(1, N - j):
                C[loc(j) + t] = C[loc(j) + t] @ Linv.conj().T
            if j + 1 < j1:  # workgroup -> tile (i, l) as ooc_pass_kernel maps it
                for blk in range(col_off(j1) - col_off(j + 1)):
                    b, l = blk, j + 1
                    while l < j1 - 1 and b >= N - l:
                        b -= N - l
                        l += 1
                    i = l + b
                    assert i < N and loc(l) + (i - l) == loc(j + 1) + blk
                    C[loc(l) + i - l] = C[loc(l) + i - l] - C[loc(j) + i - j] @ C[loc(j) + l - j].conj().T
        for t in range(nt):
            done[col_off(j0) + t] = C[t]
        # write-back: rows j1 .. N-1 of the pass's columns, the only part later passes read
        if j1 < N:
            for j in range(j0, j1):
                for r in range(j1 - j, N - j):
                    Lh[col_off(j) + r] = C[col_off(j) - col_off(j0) + r]
    L = np.zeros((npad, npad), complex)
    for k in range(N):
        for i in range(k, N):
            L[i * bs:(i + 1) * bs, k * bs:(k + 1) * bs] = done[col_off(k) + i - k]
    return np.tril(L), np.linalg.cholesky(S)


@pytest.mark.parametrize("n,avail", [(40, 20), (40, 25), (40, 60), (37, 100), (8, 4), (4, 2), (64, 32), (40, 75),
                                     (64, 150), (61, 260)])
def test_schedule_reproduces_cholesky(n, avail):
    L, ref = _schedule(n, avail)
    assert np.max(np.abs(L - ref)) <= 1e-13 * np.max(np.abs(ref))
