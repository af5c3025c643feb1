"""Seeded synthetic inputs for the histogram path (shared by the oracle tests and the HIP path).

This module only draws bytes; it holds none of the method's arithmetic.  Every
array comes from ``numpy.random.Generator(PCG64(SeedSequence([ROOT_SEED,
config, item])))`` so that a (config, item) pair names its bytes exactly.

The workloads follow the paper's shapes: 8-bit pixels, 1024x1024 and
8192x8192 slices, the four Table 2 input types (random, sequential, all equal
to 127, all equal to 1), normally distributed "X-ray-like" data, a degenerate
plus random-homogeneous mixture (Sec. III.C), and chunked streams
(Sec. III.B).  The paper's X-ray dataset is not available; the clipped
discretised Normal streams stand in for it.
"""

from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass
from typing import Iterator, List, Sequence, Tuple

import numpy as np

ROOT_SEED = 10110235
MIB = 1 << 20

# config ids (the workload families)
CFG_IMAGE = 1      # one 1024x1024 uniform image; Table 2 matrix
CFG_STREAM = 2     # single stream of 4 MiB chunks
CFG_XRAY = 3       # drifting X-ray-like frame stream
CFG_BATCH = 4      # batch of uneven images
CFG_SERVE = 5      # served requests


def rng(config: int, item: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, int(config), int(item)])))


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8).tobytes()).hexdigest()


# ----------------------------------------------------------------------------
# elementary distributions
# ----------------------------------------------------------------------------

def uniform_bytes(n: int, g: np.random.Generator) -> np.ndarray:
    return g.integers(0, 256, size=n, dtype=np.uint8)


def ramp_bytes(n: int) -> np.ndarray:
    """The 'sequential' input: in[i] = i mod 256."""
    return (np.arange(n, dtype=np.uint64) % 256).astype(np.uint8)


def constant_bytes(n: int, v: int) -> np.ndarray:
    return np.full(n, v, dtype=np.uint8)


def clipped_normal_bytes(n: int, mu: float, sigma: float, g: np.random.Generator) -> np.ndarray:
    """clip(rint(mu + sigma z), 0, 255) as uint8 (rint rounds half to even)."""
    out = np.empty(n, dtype=np.uint8)
    step = 1 << 22
    for s in range(0, n, step):
        e = min(n, s + step)
        z = g.standard_normal(e - s)
        out[s:e] = np.clip(np.rint(mu + sigma * z), 0, 255).astype(np.uint8)
    return out


def two_spike_bytes(n: int, g: np.random.Generator, lo: int = 0, hi: int = 255) -> np.ndarray:
    """Exactly n//2 bytes equal lo and n - n//2 equal hi, in a seeded random order."""
    a = np.full(n, hi, dtype=np.uint8)
    a[: n // 2] = lo
    g.shuffle(a)
    return a


def mixture_bytes(n: int, d: float, v: int, g: np.random.Generator) -> np.ndarray:
    """Degenerate + random-homogeneous mixture: exactly round(d n) positions (seeded) set to v, the rest uniform."""
    a = uniform_bytes(n, g)
    k = int(round(d * n))
    if k:
        idx = g.choice(n, size=k, replace=False)
        a[idx] = v
    return a


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def image_1mib() -> np.ndarray:
    """One 1024x1024 image of i.i.d. uniform bytes."""
    return uniform_bytes(1024 * 1024, rng(CFG_IMAGE, 0))


TABLE2_KINDS = ("random", "sequential", "all127", "all1", "xray")


def table2_input(kind: str, n: int = 8192 * 8192) -> np.ndarray:
    """The paper's Table 2 input types at an 8192x8192 slice (the X-ray column: Normal(128, 24) stand-in)."""
    if kind == "random":
        return uniform_bytes(n, rng(CFG_IMAGE, 1))
    if kind == "sequential":
        return ramp_bytes(n)
    if kind == "all127":
        return constant_bytes(n, 127)
    if kind == "all1":
        return constant_bytes(n, 1)
    if kind == "xray":
        return clipped_normal_bytes(n, 128.0, 24.0, rng(CFG_IMAGE, 2))
    raise ValueError(kind)


@dataclass(frozen=True)
class ChunkSpec:
    kind: str          # "normal", "degenerate", "twospike"
    sigma: float = 0.0
    value: int = 127


def stream_specs() -> List[ChunkSpec]:
    """The single stream's chunk order: 16 x sigma 96, 16 x sigma 32, one all-127 chunk, 16 x sigma 8, one two-spike chunk, 16 x sigma 2."""
    specs: List[ChunkSpec] = []
    specs += [ChunkSpec("normal", 96.0)] * 16
    specs += [ChunkSpec("normal", 32.0)] * 16
    specs += [ChunkSpec("degenerate", value=127)]
    specs += [ChunkSpec("normal", 8.0)] * 16
    specs += [ChunkSpec("twospike")]
    specs += [ChunkSpec("normal", 2.0)] * 16
    return specs


def stream_chunk(k: int, spec: ChunkSpec, chunk_bytes: int = 4 * MIB) -> np.ndarray:
    g = rng(CFG_STREAM, k)
    if spec.kind == "normal":
        return clipped_normal_bytes(chunk_bytes, 128.0, spec.sigma, g)
    if spec.kind == "degenerate":
        return constant_bytes(chunk_bytes, spec.value)
    if spec.kind == "twospike":
        return two_spike_bytes(chunk_bytes, g)
    raise ValueError(spec.kind)


def stream_chunks(chunk_bytes: int = 4 * MIB, count: int = None) -> List[np.ndarray]:
    specs = stream_specs()
    if count is not None:
        specs = specs[:count]
    return [stream_chunk(k, s, chunk_bytes) for k, s in enumerate(specs)]


@dataclass(frozen=True)
class FrameSpec:
    mu: float
    sigma: float


def xray_specs(count: int = 512) -> List[FrameSpec]:
    """X-ray-like frames: the mean walks mu_t = clip(mu_{t-1} + 4 N(0,1), 0, 255) from 128; sigma_t ~ U[6, 40]."""
    g = rng(CFG_XRAY, 0)
    mu = 128.0
    out = []
    for _ in range(count):
        mu = float(np.clip(mu + 4.0 * g.standard_normal(), 0.0, 255.0))
        sigma = float(g.uniform(6.0, 40.0))
        out.append(FrameSpec(mu, sigma))
    return out


def xray_frame(t: int, spec: FrameSpec, frame_bytes: int = 2048 * 2048, saturated: float = 0.01) -> np.ndarray:
    """One frame: clipped Normal(mu_t, sigma_t) with exactly round(0.01 n) seeded positions saturated at 255."""
    g = rng(CFG_XRAY, 1 + t)
    a = clipped_normal_bytes(frame_bytes, spec.mu, spec.sigma, g)
    k = int(round(saturated * frame_bytes))
    if k:
        a[g.choice(frame_bytes, size=k, replace=False)] = 255
    return a


@dataclass(frozen=True)
class ImageSpec:
    w: int
    h: int
    kind: str          # "uniform", "normal", "spike"
    mu: float = 0.0
    sigma: float = 0.0
    value: int = 0

    @property
    def size(self) -> int:
        return self.w * self.h


def batch_specs(count: int = 4096, side_lo: int = 64, side_hi: int = 4096) -> List[ImageSpec]:
    """Batch images: sides independent round(exp(U[ln lo, ln hi])); distribution uniform / Normal / 90% spike, 1/3 each."""
    g = rng(CFG_BATCH, 0)
    out = []
    for _ in range(count):
        w = int(round(math.exp(g.uniform(math.log(side_lo), math.log(side_hi)))))
        h = int(round(math.exp(g.uniform(math.log(side_lo), math.log(side_hi)))))
        kind = ("uniform", "normal", "spike")[int(g.integers(0, 3))]
        if kind == "normal":
            out.append(ImageSpec(w, h, kind, mu=float(g.uniform(20, 235)), sigma=float(g.uniform(2, 50))))
        elif kind == "spike":
            out.append(ImageSpec(w, h, kind, value=int(g.integers(0, 256))))
        else:
            out.append(ImageSpec(w, h, kind))
    return out


def batch_image(j: int, spec: ImageSpec) -> np.ndarray:
    g = rng(CFG_BATCH, 1 + j)
    n = spec.size
    if spec.kind == "uniform":
        return uniform_bytes(n, g)
    if spec.kind == "normal":
        return clipped_normal_bytes(n, spec.mu, spec.sigma, g)
    return mixture_bytes(n, 0.9, spec.value, g)


def batch_arena(specs: Sequence[ImageSpec], align: int = 256, first: int = 0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Pack images into one arena at `align`-byte aligned starts (align=1: byte-packed).

    Returns (arena uint8, offsets uint64, sizes uint64)."""
    sizes = np.array([s.size for s in specs], dtype=np.uint64)
    offsets = np.zeros(len(specs), dtype=np.uint64)
    pos = 0
    for j, s in enumerate(specs):
        pos = (pos + align - 1) // align * align
        offsets[j] = pos
        pos += s.size
    arena = np.zeros(pos, dtype=np.uint8)
    for j, s in enumerate(specs):
        o = int(offsets[j])
        arena[o:o + s.size] = batch_image(first + j, s)
    return arena, offsets, sizes


@dataclass(frozen=True)
class Request:
    t_arrival: float   # seconds from the start of the run
    size: int
    stream_id: int
    offset: int        # byte offset inside that stream's pool


def serve_requests(rate_hz: float, duration_s: float, n_streams: int = 64, size_lo: int = 4096,
                   size_hi: int = 64 * MIB, pool_bytes: int = 256 * MIB, item: int = 0) -> List[Request]:
    """Served requests: Poisson arrivals; size floor(exp(U[ln lo, ln hi])); stream id uniform; offset uniform in the pool."""
    g = rng(CFG_SERVE, item)
    out = []
    t = 0.0
    while True:
        t += float(g.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        size = int(math.floor(math.exp(g.uniform(math.log(size_lo), math.log(size_hi)))))
        size = min(size, pool_bytes)
        sid = int(g.integers(0, n_streams))
        off = int(g.integers(0, pool_bytes - size + 1))
        out.append(Request(t, size, sid, off))
    return out


def serve_pool(stream_id: int, pool_bytes: int, piece: int = 4 * MIB) -> np.ndarray:
    """A per-stream pool: consecutive drifting clipped-Normal pieces (as the X-ray frames, per stream)."""
    g = rng(CFG_SERVE, 1000 + stream_id)
    out = np.empty(pool_bytes, dtype=np.uint8)
    mu = float(g.uniform(40, 215))
    for s in range(0, pool_bytes, piece):
        e = min(pool_bytes, s + piece)
        mu = float(np.clip(mu + 4.0 * g.standard_normal(), 0.0, 255.0))
        sigma = float(g.uniform(6.0, 40.0))
        out[s:e] = clipped_normal_bytes(e - s, mu, sigma, g)
    return out


def iter_chunks(a: np.ndarray, chunk: int) -> Iterator[np.ndarray]:
    for s in range(0, a.size, chunk):
        yield a[s:s + chunk]
