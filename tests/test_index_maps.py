"""CPU emulation of the six-step FFT kernels' data movement (no GPU).

The column kernels for ny = 64 R1 (R1 = 8: 512 rows, R1 = 6: 384 rows) and
for ny = 256 on 16-column tiles, and the 384-wide row kernel, move values
between two register layouts through LDS slots.  These tests restate the
kernels' lane and slot formulas, push a
random tile through an emulated LDS array exactly as the kernels do, and
check the results against numpy's FFT; they also check that every slot map
is a bijection onto its region and that each 16-lane group of an 8-byte LDS
access hits 16 distinct slots modulo 16 (no bank conflicts).
"""
import numpy as np
import pytest


def dft(v, inv):
    """Small DFT along the last axis, unnormalised (sign + for inverse)."""
    n = v.shape[-1]
    k = np.arange(n)
    m = np.exp((1 if inv else -1) * 2j * np.pi * np.outer(k, k) / n)
    return v @ m


def tw(n, m, inv):
    return np.exp((1 if inv else -1) * 2j * np.pi * m / n)


def conflict_free(slots_per_lane):
    """slots_per_lane: (64,) slots of one wavefront instruction."""
    s = np.asarray(slots_per_lane)
    return all(len(set((s[g:g + 16] % 16).tolist())) == 16 for g in range(0, len(s), 16))


# --- column kernel: 8 columns x 64 R1 rows, 512 threads ----------------------

def col_lanes():
    tid = np.arange(512)
    wave, lane = tid // 64, tid % 64
    ca, r0 = lane & 7, 8 * wave + (lane >> 3)              # layout A
    k1, cb, u = wave, lane >> 3, lane & 7                  # layout B
    sa = 8 * r0 + (ca ^ (r0 & 7))
    sb = 512 * k1 + 8 * u + (cb ^ u)
    lw = 512 * k1 + 64 * cb
    return ca, r0, k1, cb, u, sa, sb, lw


def col_forward(tile, R1, inv):
    """tile[row, col] (64 R1 x 8) -> per-lane values x[k3] = psi(k1 + R1 u + 8 R1 k3) of column cb."""
    N = 64 * R1
    ca, r0, k1, cb, u, sa, sb, lw = col_lanes()
    xs = np.full(4096, np.nan, complex)
    x = tile[r0[:, None] + 64 * np.arange(R1)[None, :], ca[:, None]]          # (512, R1)
    x = dft(x, inv)
    x[:, 1:] *= tw(N, (r0[:, None] * np.arange(1, R1)[None, :]) % N, inv)
    for k in range(R1):
        xs[512 * k + sa] = x[:, k]
    act = k1 < R1                                                             # layout B wavefronts
    y = np.stack([xs[sb + 64 * q] for q in range(8)], axis=1)                 # (512, 8)
    y = dft(y, inv)
    y[:, 1:] *= tw(64, u[:, None] * np.arange(1, 8)[None, :], inv)
    lodd = cb & 1
    for k in range(8):
        idx = lw + 8 * (u ^ lodd) + (k ^ u)
        xs[idx[act]] = y[act, k]
    z = np.stack([xs[lw + 8 * (v ^ lodd) + (u ^ v)] for v in range(8)], axis=1)
    z = dft(z, inv)
    return z, act


@pytest.mark.parametrize("R1", [8, 6])
def test_six_step_column_forward_and_inverse(R1):
    N = 64 * R1
    rng = np.random.default_rng(R1)
    tile = rng.standard_normal((N, 8)) + 1j * rng.standard_normal((N, 8))
    ca, r0, k1, cb, u, sa, sb, lw = col_lanes()
    for inv in (False, True):
        z, act = col_forward(tile, R1, inv)
        ref = np.fft.ifft(tile, axis=0) * N if inv else np.fft.fft(tile, axis=0)
        rows = k1[:, None] + R1 * u[:, None] + 8 * R1 * np.arange(8)[None, :]
        got = z[act]
        want = ref[rows[act], cb[act][:, None]]
        assert np.allclose(got, want, rtol=0, atol=1e-9 * np.abs(ref).max())
        # every (row, column) of the tile is produced exactly once
        assert len(set(zip(rows[act].ravel().tolist(), np.repeat(cb[act], 8).tolist()))) == 8 * N


def col_retrace(z, act, R1):
    """the kernel's inverse path: lanes' x[k3] at k1 + R1 u + 8 R1 k3 -> tile rows r0 + 64 j (conjugate steps)."""
    N = 64 * R1
    ca, r0, k1, cb, u, sa, sb, lw = col_lanes()
    xs = np.full(4096, np.nan, complex)
    lodd = cb & 1
    y = dft(z, True)                                         # over k3
    for v in range(8):
        xs[(lw + 8 * (v ^ lodd) + (u ^ v))[act]] = y[act, v]
    y2 = np.zeros((512, 8), complex)
    y2[act, 0] = xs[(lw + 8 * (u ^ lodd) + u)[act]]
    for k in range(1, 8):
        y2[act, k] = xs[(lw + 8 * (u ^ lodd) + (k ^ u))[act]] * tw(64, u[act] * k, True)
    y2 = dft(y2, True)                                       # over k2: x[q] at r0 = u + 8 q
    for q in range(8):
        xs[(sb + 64 * q)[act]] = y2[act, q]
    x = np.stack([xs[512 * k + sa] for k in range(R1)], axis=1)
    x[:, 1:] *= tw(N, (r0[:, None] * np.arange(1, R1)[None, :]) % N, True)
    x = dft(x, True)
    out = np.zeros((N, 8), complex)
    out[r0[:, None] + 64 * np.arange(R1)[None, :], ca[:, None]] = x
    return out


@pytest.mark.parametrize("R1", [8, 6])
def test_six_step_column_slice_step(R1):
    # a regular slice: FFT_y, the propagator at the scrambled rows, iFFT_y
    N = 64 * R1
    rng = np.random.default_rng(10 + R1)
    tile = rng.standard_normal((N, 8)) + 1j * rng.standard_normal((N, 8))
    prop = np.exp(1j * rng.standard_normal((N, 8)))
    ca, r0, k1, cb, u, sa, sb, lw = col_lanes()
    z, act = col_forward(tile, R1, False)
    rows = k1[:, None] + R1 * u[:, None] + 8 * R1 * np.arange(8)[None, :]
    z[act] *= prop[rows[act], cb[act][:, None]]
    out = col_retrace(z, act, R1)
    want = np.fft.ifft(prop * np.fft.fft(tile, axis=0), axis=0) * N
    assert np.allclose(out, want, rtol=0, atol=1e-9 * np.abs(want).max())


@pytest.mark.parametrize("R1", [8, 6])
def test_six_step_column_slots(R1):
    ca, r0, k1, cb, u, sa, sb, lw = col_lanes()
    # cross-wavefront exchange: writes 512 k + sa (k < R1), reads sb + 64 q
    for k in range(R1):
        assert sorted((512 * k + sa).tolist()) == list(range(512 * k, 512 * k + 512))
        for w in range(8):
            assert conflict_free((512 * k + sa)[64 * w:64 * w + 64])
    for q in range(8):
        for w in range(R1):
            assert conflict_free((sb + 64 * q)[64 * w:64 * w + 64])
    reads = np.concatenate([(sb + 64 * q)[:64 * R1] for q in range(8)])
    assert sorted(reads.tolist()) == list(range(512 * R1))
    # local exchange inside wavefront k1's 512 slots
    lodd = cb & 1
    for k in range(8):
        wr = lw + 8 * (u ^ lodd) + (k ^ u)
        rd = lw + 8 * (k ^ lodd) + (u ^ k)
        for w in range(R1):
            assert conflict_free(wr[64 * w:64 * w + 64]) and conflict_free(rd[64 * w:64 * w + 64])
            assert np.all(wr[64 * w:64 * w + 64] // 512 == w)


# --- column kernel for 256 = 8 x 32 rows on 16-column tiles, 512 threads -----

def q_lanes():
    tid = np.arange(512)
    wave, lane = tid // 64, tid % 64
    ca, r0 = lane & 15, 4 * wave + (lane >> 4)             # layout A
    k1, cb, u = wave, lane >> 2, lane & 3                  # layout B
    sa = 16 * r0 + (ca ^ (4 * (r0 & 3)))
    sb = 512 * k1 + 16 * u + (cb ^ (4 * u))
    lw = 512 * k1 + 32 * cb
    cs = cb & 3
    return ca, r0, k1, cb, u, sa, sb, lw, cs


def lslot(k2, uu, cs):
    return 16 * (k2 >> 2) + 4 * ((k2 & 3) ^ cs) + (uu ^ cs)


def test_six_step_column_256_slice_step():
    N = 256
    rng = np.random.default_rng(256)
    tile = rng.standard_normal((N, 16)) + 1j * rng.standard_normal((N, 16))
    prop = np.exp(1j * rng.standard_normal((N, 16)))
    ca, r0, k1, cb, u, sa, sb, lw, cs = q_lanes()
    xs = np.full(4096, np.nan, complex)
    # forward: layout A
    x = tile[r0[:, None] + 32 * np.arange(8)[None, :], ca[:, None]]
    x = dft(x, False)
    x[:, 1:] *= tw(N, r0[:, None] * np.arange(1, 8)[None, :], False)
    for k in range(8):
        xs[512 * k + sa] = x[:, k]
    # layout B
    y = np.stack([xs[sb + 64 * q] for q in range(8)], axis=1)
    y = dft(y, False)
    y[:, 1:] *= tw(32, u[:, None] * np.arange(1, 8)[None, :], False)
    for k in range(8):
        xs[lw + lslot(k, u, cs)] = y[:, k]
    z = np.stack([xs[lw + lslot(u + 4 * (v >> 2), v & 3, cs)] for v in range(8)], axis=1)
    z = np.concatenate([dft(z[:, :4], False), dft(z[:, 4:], False)], axis=1)
    rows = np.stack([k1 + 8 * (u + 4 * (e >> 2)) + 64 * (e & 3) for e in range(8)], axis=1)
    spec = np.fft.fft(tile, axis=0)
    assert np.allclose(z, spec[rows, cb[:, None]], rtol=0, atol=1e-9 * np.abs(spec).max())
    assert len(set(zip(rows.ravel().tolist(), np.repeat(cb, 8).tolist()))) == 16 * N
    # propagator, then the inverse retraced
    z = z * prop[rows, cb[:, None]]
    z = np.concatenate([dft(z[:, :4], True), dft(z[:, 4:], True)], axis=1)
    for h in range(2):
        for v in range(4):
            xs[lw + lslot(u + 4 * h, v, cs)] = z[:, 4 * h + v]
    y = np.stack([xs[lw + lslot(k, u, cs)] for k in range(8)], axis=1)
    y[:, 1:] *= tw(32, u[:, None] * np.arange(1, 8)[None, :], True)
    y = dft(y, True)
    for q in range(8):
        xs[sb + 64 * q] = y[:, q]
    x = np.stack([xs[512 * k + sa] for k in range(8)], axis=1)
    x[:, 1:] *= tw(N, r0[:, None] * np.arange(1, 8)[None, :], True)
    x = dft(x, True)
    out = np.zeros((N, 16), complex)
    out[r0[:, None] + 32 * np.arange(8)[None, :], ca[:, None]] = x
    want = np.fft.ifft(prop * spec, axis=0) * N
    assert np.allclose(out, want, rtol=0, atol=1e-9 * np.abs(want).max())
    # bank checks: every wavefront instruction of every exchange
    for w in range(8):
        sl = slice(64 * w, 64 * w + 64)
        for k in range(8):
            assert conflict_free((512 * k + sa)[sl]) and conflict_free((lw + lslot(k, u, cs))[sl])
        for q in range(8):
            assert conflict_free((sb + 64 * q)[sl])
        for v in range(8):
            assert conflict_free((lw + lslot(u + 4 * (v >> 2), v & 3, cs))[sl])


# --- row kernel for 384 = 6 x 64, one row per wavefront ------------------------

def r6_slot(t, k):
    return 64 * k + (t ^ (8 * (k & 1)))


def row_a_to_b(x_nat, inv):
    """natural row (384) -> lanes 0-47: values at k1 + 6 u + 48 k3."""
    t = np.arange(64)
    k1, u = t >> 3, t & 7
    act = t < 48
    xs = np.full(384, np.nan, complex)
    x = x_nat[t[:, None] + 64 * np.arange(6)[None, :]]
    x = dft(x, inv)
    x[:, 1:] *= tw(384, t[:, None] * np.arange(1, 6)[None, :], inv)
    for k in range(6):
        xs[r6_slot(t, k)] = x[:, k]
    y = np.zeros((64, 8), complex)
    y[act] = np.stack([xs[r6_slot(u[act] + 8 * q, k1[act])] for q in range(8)], axis=1)
    y = dft(y, inv)
    y[:, 1:] *= tw(64, u[:, None] * np.arange(1, 8)[None, :], inv)
    lodd, lw = k1 & 1, 64 * k1
    for k in range(8):
        xs[(lw + 8 * (u ^ lodd) + (k ^ u))[act]] = y[act, k]
    z = np.zeros((64, 8), complex)
    z[act] = np.stack([xs[(lw + 8 * (v ^ lodd) + (u ^ v))[act]] for v in range(8)], axis=1)
    return dft(z, inv), act


def row_b_to_a(z, act):
    """lanes 0-47 holding g at k1 + 6 u + 48 k3 -> natural forward DFT of g."""
    t = np.arange(64)
    k1, u = t >> 3, t & 7
    xs = np.full(384, np.nan, complex)
    lodd, lw = k1 & 1, 64 * k1
    y = dft(z, False)                                   # over k3
    for w in range(8):
        xs[(lw + 8 * (w ^ lodd) + (u ^ w))[act]] = y[act, w]
    y2 = np.zeros((64, 8), complex)
    y2[act, 0] = xs[(lw + 8 * (u ^ lodd) + u)[act]]
    for k in range(1, 8):
        y2[act, k] = xs[(lw + 8 * (u ^ lodd) + (k ^ u))[act]] * tw(64, u[act] * k, False)
    y2 = dft(y2, False)                                 # over k2: x[q] at t = u + 8 q
    for q in range(8):
        xs[r6_slot(u[act] + 8 * q, k1[act])] = y2[act, q]
    x = np.stack([xs[r6_slot(t, k)] for k in range(6)], axis=1)
    x[:, 1:] *= tw(384, t[:, None] * np.arange(1, 6)[None, :], False)
    return dft(x, False)                                # out[t + 64 j] = x[:, j]


def test_six_step_row_384_paths():
    rng = np.random.default_rng(384)
    f = rng.standard_normal(384) + 1j * rng.standard_normal(384)
    t = np.arange(64)
    k1, u = t >> 3, t & 7
    pos = k1[:, None] + 6 * u[:, None] + 48 * np.arange(8)[None, :]
    scale = np.abs(np.fft.fft(f)).max()
    # forward natural -> scrambled (a first-slice row) and conjugate (a later row's inverse)
    for inv, ref in ((False, np.fft.fft(f)), (True, np.fft.ifft(f) * 384)):
        z, act = row_a_to_b(f, inv)
        assert np.allclose(z[act], ref[pos[act]], rtol=0, atol=1e-9 * scale)
    # scrambled -> natural forward (a later row's return after the transmission)
    g = rng.standard_normal(384) + 1j * rng.standard_normal(384)
    act = t < 48
    zg = np.zeros((64, 8), complex)
    zg[act] = g[pos[act]]
    out = row_b_to_a(zg, act)
    want = np.fft.fft(g)
    assert np.allclose(out, want[t[:, None] + 64 * np.arange(6)[None, :]], rtol=0,
                       atol=1e-9 * np.abs(want).max())
    # a later-slice row end to end: FFT(t(x) * IFFT(psi)) up to the 1/N the
    # propagator carries
    psi = np.fft.fft(rng.standard_normal(384) + 1j * rng.standard_normal(384))
    trans = np.exp(1j * rng.standard_normal(384))
    z, act = row_a_to_b(psi, True)
    z[act] *= trans[pos[act]]
    out = row_b_to_a(z, act)
    want = np.fft.fft(trans * np.fft.ifft(psi) * 384)
    assert np.allclose(out, want[t[:, None] + 64 * np.arange(6)[None, :]], rtol=0,
                       atol=1e-9 * np.abs(want).max())


def test_six_step_row_384_slots():
    t = np.arange(64)
    k1, u = t >> 3, t & 7
    act = t < 48
    slots = np.array([[r6_slot(tt, k) for k in range(6)] for tt in t])
    assert sorted(slots.ravel().tolist()) == list(range(384))
    for k in range(6):
        assert conflict_free(slots[:, k])
    for q in range(8):
        rd = np.array([r6_slot(int(uu) + 8 * q, int(kk)) for uu, kk in zip(u, k1)])
        assert all(len(set((rd[act][g:g + 16] % 16).tolist())) == 16 for g in range(0, 48, 16))
    lodd, lw = k1 & 1, 64 * k1
    for k in range(8):
        wr = (lw + 8 * (u ^ lodd) + (k ^ u))[act]
        assert all(len(set((wr[g:g + 16] % 16).tolist())) == 16 for g in range(0, 48, 16))
        assert np.all(wr // 64 == k1[act])
