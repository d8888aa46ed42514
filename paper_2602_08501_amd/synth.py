"""Seeded synthetic workload: transmitter and AWGN channel.

This module produces the decoder's inputs and nothing else.  It holds none
of the decoder's arithmetic (no list decoding, no move search) and is the
only module that both the HIP path and the test oracle consume.

Transmitter and channel (Sec. II-B of the paper): a uniformly random payload
of ``k_pay`` bits is extended by a CRC of ``crc_len`` bits (v = payload ||
crc), v is placed on the information positions of RM(r, m) (ascending), the
codeword is c = u F^{(x)m}, the BPSK symbols are x = 1 - 2c and the channel
adds white Gaussian noise of variance sigma^2 = N0 / 2 with
    sigma^2 = 1 / (2 R 10^(EbN0/10)),   R = k_pay / N.
The received values are rounded once to float32.

Random numbers come from a counter-based SplitMix64 generator (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
the k-th output of stream kappa is mix64(kappa + (k + 1) * GAMMA).  Every
frame has its own stream keyed by (seed, workload id, SNR index, frame
index), so a frame's data does not depend on the batch it is generated in.
Gaussian samples use the Box-Muller transform on 53-bit uniforms.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

CRC6_POLY = 0x43  # x^6 + x + 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on uint64 arrays (wrap-around arithmetic)."""
    z = np.asarray(z, np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(base: np.ndarray, x) -> np.ndarray:
    with np.errstate(over="ignore"):
        return mix64(np.asarray(base, np.uint64) ^ mix64((np.asarray(x, np.uint64) + np.uint64(1)) * GAMMA))


def stream_keys(seed: int, workload: int, snr_index: int, frames: np.ndarray, purpose: int) -> np.ndarray:
    k = mix64(np.array([(seed * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019) & _MASK64], np.uint64))
    k = _key(k, workload)
    k = _key(k, snr_index)
    k = _key(k, np.asarray(frames, np.uint64))
    return _key(k, purpose)


def stream(keys: np.ndarray, count: int) -> np.ndarray:
    """[len(keys)][count] uint64: outputs 0..count-1 of each stream."""
    ctr = (np.arange(1, count + 1, dtype=np.uint64))[None, :]
    with np.errstate(over="ignore"):
        return mix64(keys[:, None] + ctr * GAMMA)


def uniform53(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def gaussian(keys: np.ndarray, n: int) -> np.ndarray:
    """[len(keys)][n] standard normal samples (n even), Box-Muller."""
    assert n % 2 == 0
    u = uniform53(stream(keys, n))
    u1, u2 = u[:, 0::2], u[:, 1::2]
    rad = np.sqrt(-2.0 * np.log1p(-u1))
    ang = 2.0 * math.pi * u2
    out = np.empty((len(keys), n), np.float64)
    out[:, 0::2] = rad * np.cos(ang)
    out[:, 1::2] = rad * np.sin(ang)
    return out


# ------------------------------------------------------------------ transmitter
def info_positions(r: int, m: int) -> np.ndarray:
    """Rows of F^{(x)m} spanning RM(r, m): popcount(i) >= m - r, ascending."""
    idx = np.arange(1 << m)
    pc = np.array([bin(i).count("1") for i in idx])
    return idx[pc >= m - r]


def crc_append(payload: np.ndarray, crc_len: int, poly: int) -> np.ndarray:
    """[F][k] bits -> [F][k + crc_len]: remainder of p(x) x^L mod g(x), first
    bit highest degree, non-reflected, init 0."""
    F, k = payload.shape
    if crc_len == 0:
        return payload.copy()
    reg = np.zeros(F, np.uint32)
    top, mask = np.uint32(1 << (crc_len - 1)), np.uint32((1 << crc_len) - 1)
    low = np.uint32(poly & ((1 << crc_len) - 1))
    for i in range(k):
        fb = ((reg & top) != 0).astype(np.uint32) ^ payload[:, i].astype(np.uint32)
        reg = (reg << np.uint32(1)) & mask
        reg ^= fb * low
    crc = np.stack([(reg >> np.uint32(crc_len - 1 - t)) & np.uint32(1) for t in range(crc_len)], 1)
    return np.concatenate([payload, crc.astype(np.uint8)], 1)


def polar_transform(u: np.ndarray, m: int) -> np.ndarray:
    """c = u F^{(x)m} over GF(2), row-wise on [F][N] bits."""
    c = u.copy()
    n = 1 << m
    for s in range(m):
        h = 1 << s
        c = c.reshape(-1, n // (2 * h), 2, h)
        c[:, :, 0, :] ^= c[:, :, 1, :]
        c = c.reshape(-1, n)
    return c


@dataclasses.dataclass(frozen=True)
class Workload:
    """One code / SNR point.  ``wid`` names the workload in the RNG key."""
    r: int
    m: int
    k_pay: int
    crc_len: int = 6
    crc_poly: int = CRC6_POLY
    ebn0_db: float = 2.5
    wid: int = 1
    snr_index: int = 0

    @property
    def N(self) -> int:
        return 1 << self.m

    @property
    def rate(self) -> float:
        return self.k_pay / self.N

    @property
    def sigma2(self) -> float:
        return 1.0 / (2.0 * self.rate * 10.0 ** (self.ebn0_db / 10.0))

    @property
    def llr_scale(self) -> np.float32:
        """Quantizer scale 8 / sigma^2 (four times the LLR 2y/sigma^2), as float32."""
        return np.float32(8.0 / self.sigma2)


def generate(wl: Workload, seed: int, f0: int, f1: int):
    """Frames [f0, f1): (payload bits, transmitted codeword bits, y float32)."""
    frames = np.arange(f0, f1, dtype=np.uint64)
    F, n = len(frames), wl.N
    kp = stream_keys(seed, wl.wid, wl.snr_index, frames, 0)
    payload = (stream(kp, wl.k_pay) >> np.uint64(63)).astype(np.uint8)
    v = crc_append(payload, wl.crc_len, wl.crc_poly)
    A = info_positions(wl.r, wl.m)
    if v.shape[1] != len(A):
        raise ValueError("payload + CRC must fill the %d information positions" % len(A))
    u = np.zeros((F, n), np.uint8)
    u[:, A] = v
    c = polar_transform(u, wl.m)
    kn = stream_keys(seed, wl.wid, wl.snr_index, frames, 1)
    noise = gaussian(kn, n) * math.sqrt(wl.sigma2)
    y = ((1.0 - 2.0 * c.astype(np.float64)) + noise).astype(np.float32)
    return payload, c, y


def generate_snr_mix(wl: Workload, seed: int, f0: int, f1: int, ebn0_lo: float, ebn0_hi: float):
    """Frames [f0, f1) whose Eb/N0 is drawn per frame uniformly in
    [ebn0_lo, ebn0_hi] (from the frame's own stream).  Returns (payload,
    codeword, y float32, per-frame Eb/N0, per-frame quantizer scale 8/sigma^2
    as float32)."""
    frames = np.arange(f0, f1, dtype=np.uint64)
    F, n = len(frames), wl.N
    kp = stream_keys(seed, wl.wid, wl.snr_index, frames, 0)
    payload = (stream(kp, wl.k_pay) >> np.uint64(63)).astype(np.uint8)
    v = crc_append(payload, wl.crc_len, wl.crc_poly)
    A = info_positions(wl.r, wl.m)
    u = np.zeros((F, n), np.uint8)
    u[:, A] = v
    c = polar_transform(u, wl.m)
    ks = stream_keys(seed, wl.wid, wl.snr_index, frames, 2)
    ebn0 = ebn0_lo + (ebn0_hi - ebn0_lo) * uniform53(stream(ks, 1)[:, 0])
    sigma2 = 1.0 / (2.0 * wl.rate * 10.0 ** (ebn0 / 10.0))
    kn = stream_keys(seed, wl.wid, wl.snr_index, frames, 1)
    noise = gaussian(kn, n) * np.sqrt(sigma2)[:, None]
    y = ((1.0 - 2.0 * c.astype(np.float64)) + noise).astype(np.float32)
    return payload, c, y, ebn0, (8.0 / sigma2).astype(np.float32)


# The workloads the decoder is measured on (codes, payloads and SNR grids).
RM26 = Workload(r=2, m=6, k_pay=16, ebn0_db=3.0, wid=0)
RM37 = Workload(r=3, m=7, k_pay=58, ebn0_db=2.5, wid=1)
RM27 = Workload(r=2, m=7, k_pay=23, ebn0_db=2.5, wid=2)
RM38 = Workload(r=3, m=8, k_pay=87, ebn0_db=2.0, wid=3)
