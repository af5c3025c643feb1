"""CPU oracle for the adaptive-histogram hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP path and
never imports the ``paper_1011_0235_amd`` package.

Contents, each written from the paper (Koppaka et al., "Fast Histograms using
Adaptive CUDA Streams", 2010):

* ``hist`` / ``hist_py`` -- the exact 256-bin histogram of packed 8-bit pixels
  (Sec. III.A: pixels are bytes with values 0..255; the block output is the
  256-INT histogram; Sec. I: the problem is exact histogram computation).
  ``hist`` runs the plain C counting loop of ``oracle.c``; ``hist_py`` is a
  pure-Python twin for tiny inputs.
* The binning pattern (Sec. III.A, Figure 1 -- the figure itself is missing
  from the text): 256 entries, one per pixel value, naming that value's
  sub-bins in the shared sub-histogram.  Encoding (our reading): one 32-bit
  word per value, bits [0,16) = base sub-bin, bits [16,24) = log2(r), r a power
  of two.  Lane L of a wavefront adds into sub-bin base + (L mod r): the paper
  allots sub-bins to the threads of a warp cyclically (Sec. III.A, discussion
  of Table 2).
* ``pattern_paper960`` -- our reconstruction of the paper's own pattern: length
  960, eight sub-bins for value 127 (the most), one sub-bin for the first bin
  (Sec. III.A and the discussion of Table 2).  Only those facts pin it;
  everything else about it is PARITY UNPINNED.
* ``rule_p`` -- recomputing the pattern from past histograms (Sec. III.B says
  the indices are recomputed from the past stream's histograms but gives no
  rule).  Rule P below is our reading; it is pinned by closed forms and
  structural invariants only (PARITY UNPINNED against the paper).
* ``is_degenerate`` -- the degeneracy criterion (Sec. III.C): switch to AHist
  when any bin of the last moving-window histogram exceeds the critical
  degeneracy (40-50 %); tested exactly in integers as 100*max > theta*sum.
* ``collision_index`` / ``collides`` -- an alternative switching criterion (the paper
  leaves other criteria to future work and names one that measures the serialisation the
  data would cause): the probability sum_v p_v^2 that two lanes add into the same bin,
  compared with kappa.  Our reading; pinned by closed forms and invariants
  (tests/test_criterion_cpu.py).
* ``change_alarm`` -- change detection (Sec. III.B: the moving window, the stream's
  present, compared with the Accumulator, its general nature, to detect an attack or a
  need to reprocess).  The paper fixes no measure; our reading: alarm when some value's
  share of the window differs from its share of the Accumulator by more than alarm_pct
  percentage points (strict), computed with exact fractions.  Pinned by hand-worked
  examples, a closed form and invariants (tests/test_change_cpu.py).
* ``stream_reference`` -- Accumulator and moving-window (MW) histograms of a
  chunked stream and the kernel/pattern decision carried from chunk to chunk
  (Sec. III.B, Sec. III.C), with a pipeline lag (Sec. III.B, Figure 2: the
  CPU prepares the next iteration while the GPU runs the current one).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

MODE_AUTO = 0
MODE_AHIST = 1
MODE_WAVEHIST = 2
MODE_WAVEAGG = 3      # a forced-only kernel choice; the switch itself picks AHist or per-wavefront

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_oracle(force: bool = False) -> str:
    """Compile oracle.c with gcc -O2 (no intrinsics) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_oracle()
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_hist_u8.argtypes = [u8p, ctypes.c_size_t, u64p]
        lib.oracle_hist_u8.restype = None
        lib.oracle_hist_u8_acc.argtypes = [u8p, ctypes.c_size_t, u64p]
        lib.oracle_hist_u8_acc.restype = None
        lib.oracle_hist_many.argtypes = [u8p, u64p, u64p, ctypes.c_size_t, u64p]
        lib.oracle_hist_many.restype = None
        lib.oracle_hist_timed.argtypes = [u8p, ctypes.c_size_t, ctypes.c_int, u64p]
        lib.oracle_hist_timed.restype = ctypes.c_double
        _lib = lib
    return _lib


def _u8(data) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(data, dtype=np.uint8).reshape(-1))
    return a


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ----------------------------------------------------------------------------
# The histogram (Sec. III.A; exactness: Sec. I)
# ----------------------------------------------------------------------------

def hist_py(data: Iterable[int]) -> List[int]:
    """Pure-Python counting loop: out[b] = #{i : data[i] == b}.  Tiny inputs only."""
    out = [0] * 256
    for v in data:
        out[int(v)] += 1
    return out


def hist(data) -> np.ndarray:
    """Exact histogram by the C counting loop; returns uint64[256]."""
    a = _u8(data)
    out = np.zeros(256, dtype=np.uint64)
    _load().oracle_hist_u8(_ptr(a, ctypes.c_uint8), a.size, _ptr(out, ctypes.c_uint64))
    return out


def hist_many(arena, offsets: Sequence[int], sizes: Sequence[int]) -> np.ndarray:
    """Histogram of each arena[offsets[j] : offsets[j] + sizes[j]]; returns uint64[count, 256]."""
    a = _u8(arena)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    sz = np.ascontiguousarray(np.asarray(sizes, dtype=np.uint64))
    if off.size != sz.size:
        raise ValueError("offsets and sizes differ in length")
    if off.size and int((off + sz).max()) > a.size:
        raise ValueError("a buffer runs past the arena")
    out = np.zeros((off.size, 256), dtype=np.uint64)
    _load().oracle_hist_many(_ptr(a, ctypes.c_uint8), _ptr(off, ctypes.c_uint64),
                             _ptr(sz, ctypes.c_uint64), off.size, _ptr(out, ctypes.c_uint64))
    return out


def hist_timed(data, threads: int):
    """(seconds, uint64[256]) for the plain loop split over `threads` contiguous slices."""
    a = _u8(data)
    out = np.zeros(256, dtype=np.uint64)
    t = _load().oracle_hist_timed(_ptr(a, ctypes.c_uint8), a.size, int(threads), _ptr(out, ctypes.c_uint64))
    if t < 0:
        raise RuntimeError("oracle timing: could not start all threads")
    return t, out


# ----------------------------------------------------------------------------
# Binning pattern (Sec. III.A, Figure 1; encoding is our reading)
# ----------------------------------------------------------------------------

def pat_word(base: int, r: int) -> int:
    """Encode one value's sub-bin range: base in bits [0,16), log2(r) in bits [16,24)."""
    if r < 1 or r & (r - 1):
        raise ValueError("r must be a power of two")
    if not 0 <= base < (1 << 16):
        raise ValueError("base out of range")
    return base | ((r.bit_length() - 1) << 16)


def pat_base(word: int) -> int:
    return int(word) & 0xFFFF


def pat_r(word: int) -> int:
    return 1 << ((int(word) >> 16) & 0xFF)


def pattern_from_r(r: Sequence[int], order: Optional[Sequence[int]] = None) -> List[int]:
    """Lay the values out contiguously in `order` (default: value order); base = running sum of r."""
    if order is None:
        order = range(256)
    words = [0] * 256
    base = 0
    for b in order:
        words[b] = pat_word(base, int(r[b]))
        base += int(r[b])
    return words


def pattern_identity() -> List[int]:
    """r = 1 for every value, base[b] = b, S = 256 (a plain shared 256-bin table)."""
    return pattern_from_r([1] * 256)


def pattern_flat(r: int) -> List[int]:
    """Every value gets r sub-bins, laid out in value order (S = 256 r)."""
    return pattern_from_r([r] * 256)


def paper960_r() -> List[int]:
    """Our reconstruction of Figure 1: eight runs of 32 values with r = 1,2,4,8,8,4,2,1.

    Pinned facts (Sec. III.A and the discussion of Table 2): length 960; value
    127 has the most sub-bins, eight; the first bin has a single sub-bin.  The
    shape of the remaining runs is PARITY UNPINNED.
    """
    runs = [1, 2, 4, 8, 8, 4, 2, 1]
    return [runs[b // 32] for b in range(256)]


def pattern_paper960() -> List[int]:
    return pattern_from_r(paper960_r())


def pattern_total(words: Sequence[int]) -> int:
    """Smallest S holding every range [base, base + r)."""
    return max(pat_base(w) + pat_r(w) for w in words)


def pattern_valid(words: Sequence[int], S: int, rmax: int) -> bool:
    """Valid iff every r is a power of two in [1, rmax], ranges lie in [0, S) and are pairwise disjoint."""
    if len(words) != 256:
        return False
    if rmax < 1 or rmax & (rmax - 1):
        return False
    used = [False] * S
    for w in words:
        w = int(w)
        if w >> 24:
            return False
        base, r = pat_base(w), pat_r(w)
        if r > rmax or base + r > S:
            return False
        for s in range(base, base + r):
            if used[s]:
                return False
            used[s] = True
    return True


def _ceil_div(a: int, b: int) -> int:
    """ceil(a / b) for integers a >= 0, b > 0 (exact, no floating point)."""
    return -(-a // b)


def _pow2ceil(x: int) -> int:
    p = 1
    while p < x:
        p <<= 1
    return p


def rule_p(h: Sequence[int], S: int, rmax: int, T: int = 24) -> List[int]:
    """Rule P: a pattern from a past histogram h (our reading; the paper gives no rule).

    0. If the budget holds rmax sub-bins for every value (256 * rmax <= S), every
       value gets rmax: the pattern exists to share a limited sub-histogram
       (Sec. III.A), and with room for all there is nothing to share.
    1. N = sum h.  N = 0 -> every r = 1.
    2. For t = 0..T' (T' = min(T, 64 - bitlen(N)), so h * 2**t stays below 2**64):
       r_t[b] = min(rmax, pow2ceil(max(1, ceil(h[b] * 2**t / N)))).
    3. Keep the largest t with sum_b r_t[b] <= S (r_0 = 1 everywhere, so t = 0
       qualifies whenever S >= 256).
    4. Lay values out by (r descending, value ascending); bases are running
       sums, so each base is a multiple of its r.
    """
    h = [int(x) for x in h]
    if len(h) != 256:
        raise ValueError("h must have 256 entries")
    if S < 256 or rmax < 1 or rmax & (rmax - 1):
        raise ValueError("need S >= 256 and rmax a power of two")
    N = sum(h)
    if 256 * rmax <= S:
        r = [rmax] * 256
    elif N == 0:
        r = [1] * 256
    else:
        tmax = min(T, 64 - N.bit_length())
        r = [1] * 256
        for t in range(0, tmax + 1):
            rt = [min(rmax, _pow2ceil(max(1, _ceil_div(hb << t, N)))) for hb in h]
            if sum(rt) <= S:
                r = rt
            else:
                break
    order = sorted(range(256), key=lambda b: (-r[b], b))
    return pattern_from_r(r, order)


# ----------------------------------------------------------------------------
# Degeneracy criterion and kernel switching (Sec. III.C)
# ----------------------------------------------------------------------------

def is_degenerate(mw: Sequence[int], theta_pct: int) -> bool:
    """True iff some bin exceeds theta percent of the window: 100 * max(mw) > theta * sum(mw)."""
    mw = [int(x) for x in mw]
    return 100 * max(mw) > int(theta_pct) * sum(mw)


def decide_mode(mw: Sequence[int], theta_pct: int, criterion: int = 0, kappa_pct: int = 0) -> int:
    """AHist when the moving-window histogram calls for it, the per-wavefront kernel otherwise.

    criterion 0 (CRIT_MAXBIN): the paper's degeneracy test, some bin above theta percent.
    criterion 1 (CRIT_COLLISION): the alternative criterion, the collision index above kappa.
    criterion 2 (CRIT_BOTH): either (the paper suggests combining the two kinds of test)."""
    deg = is_degenerate(mw, theta_pct)
    if criterion == CRIT_MAXBIN:
        ahist = deg
    elif criterion == CRIT_COLLISION:
        ahist = collides(mw, kappa_pct)
    elif criterion == CRIT_BOTH:
        ahist = deg or collides(mw, kappa_pct)
    else:
        raise ValueError("unknown criterion")
    return MODE_AHIST if ahist else MODE_WAVEHIST


# ----------------------------------------------------------------------------
# An alternative switching criterion (Sec. IV: future work)
# ----------------------------------------------------------------------------

CRIT_MAXBIN = 0
CRIT_COLLISION = 1
CRIT_BOTH = 2


def collision_index(mw: Sequence[int]):
    """Probability that two bytes drawn independently from the window's distribution are equal,
    sum_v p_v^2 with p_v = mw(v) / sum(mw), as an exact fraction (0 for an empty window).

    The paper leaves other switching criteria to future work and names one that measures the
    serialisation the data would cause.  The per-wavefront kernel serialises when lanes of a
    wavefront add into the same bin at once; for bytes drawn from p, two given lanes do so with
    probability sum_v p_v^2, so this index is our reading of that criterion."""
    from fractions import Fraction
    mw = [int(x) for x in mw]
    n = sum(mw)
    if n == 0:
        return Fraction(0)
    return Fraction(sum(x * x for x in mw), n * n)


def collides(mw: Sequence[int], kappa_pct: int) -> bool:
    """The alternative criterion: the collision index exceeds kappa percent (strict)."""
    from fractions import Fraction
    return collision_index(mw) > Fraction(int(kappa_pct), 100)


# ----------------------------------------------------------------------------
# Change detection: the moving window against the Accumulator (Sec. III.B)
# ----------------------------------------------------------------------------

def share_departure(mw: Sequence[int], acc: Sequence[int]):
    """Largest difference, over the 256 values, between a value's share of the window and its
    share of the Accumulator, as an exact fraction (0 when either histogram is empty)."""
    from fractions import Fraction
    mw, acc = [int(x) for x in mw], [int(x) for x in acc]   # exact (numpy integers would wrap)
    n_mw, n_acc = sum(mw), sum(acc)
    if n_mw == 0 or n_acc == 0:
        return Fraction(0)
    return max(abs(Fraction(m, n_mw) - Fraction(a, n_acc)) for m, a in zip(mw, acc))


def change_alarm(mw: Sequence[int], acc: Sequence[int], alarm_pct: int) -> bool:
    """Our reading of the comparison the paper proposes (the window, the stream's present, set
    against the Accumulator, its general nature, to detect an attack or a need to reprocess;
    the paper fixes no measure): alarm iff some value's share of the window differs from its
    share of the Accumulator by more than alarm_pct percentage points (strict).  Off when
    alarm_pct is 0 or either histogram is empty."""
    if alarm_pct == 0:
        return False
    from fractions import Fraction
    return share_departure(mw, acc) > Fraction(alarm_pct, 100)


# ----------------------------------------------------------------------------
# Stream semantics (Sec. III.B: Accumulator and MW; Sec. III.C: switching)
# ----------------------------------------------------------------------------

def stream_reference(chunks: Sequence, W: int = 1, theta_pct: int = 45, S: int = 960,
                     rmax: int = 8, lag: int = 0, mode: int = MODE_AUTO,
                     hists: Optional[Sequence[Sequence[int]]] = None,
                     alarm_pct: int = 0, criterion: int = CRIT_MAXBIN, kappa_pct: int = 0) -> Dict[str, object]:
    """Run a chunked stream through the adaptive scheme; return every per-chunk quantity.

    Chunk k gets histogram h_k.  After chunk k:
      Acc_k = Acc_{k-1} + h_k                                     (Accumulator)
      MW_k  = h_{max(0,k-W+1)} + ... + h_k                        (moving window of W chunks)
      D_k   = (AHIST if degenerate(MW_k) else WAVEHIST, rule_p(MW_k))
    Chunk k runs with D_{k-1-lag}; chunks with k - 1 - lag < 0 have no history and
    run the per-wavefront kernel with the identity pattern.  A forced mode
    (AHIST / WAVEHIST) replaces the decided kernel but not the pattern.

    With alarm_pct > 0, A_k = change_alarm(MW_k, Acc_k, alarm_pct) after every chunk.
    `criterion` / `kappa_pct` choose the switching test (see decide_mode).

    `hists` may pass precomputed chunk histograms (from ``hist``) to skip recounting.
    Returns dict with keys: hists (uint64[k,256]), acc (int list), mw (int list,
    after the last chunk), modes (kernel used per chunk), patterns (pattern used
    per chunk, 256 words each), alarms (0/1 per chunk).
    """
    if W < 1 or lag < 0:
        raise ValueError("need W >= 1 and lag >= 0")
    nchunk = len(chunks) if hists is None else len(hists)
    hs = [list(map(int, hist(c))) for c in chunks] if hists is None else [list(map(int, x)) for x in hists]
    acc = [0] * 256
    decisions = []
    modes: List[int] = []
    patterns: List[List[int]] = []
    mw = [0] * 256
    alarms: List[int] = []
    for k in range(nchunk):
        j = k - 1 - lag
        if j >= 0:
            dec_mode, dec_pat = decisions[j]
        else:
            dec_mode, dec_pat = MODE_WAVEHIST, pattern_identity()
        modes.append(dec_mode if mode == MODE_AUTO else mode)
        patterns.append(list(dec_pat))
        acc = [a + b for a, b in zip(acc, hs[k])]
        lo = max(0, k - W + 1)
        mw = [sum(hs[i][b] for i in range(lo, k + 1)) for b in range(256)]
        decisions.append((decide_mode(mw, theta_pct, criterion, kappa_pct), rule_p(mw, S, rmax)))
        alarms.append(1 if change_alarm(mw, acc, alarm_pct) else 0)
    return {
        "hists": np.array(hs, dtype=np.uint64).reshape(nchunk, 256),
        "acc": acc,
        "mw": mw,
        "modes": modes,
        "patterns": patterns,
        "alarms": alarms,
    }
