"""Counter-based random streams for the synthetic inputs.

Every random number is a pure function of (seed, stream, index), so any
slice of any stream can be produced in any order and on any machine with
the same result.  The mixing function is the SplitMix64 finaliser
(G. L. Steele, D. Lea, C. H. Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014, with the output constants of D. Stafford's
"Mix13").  Normal variates use the Box-Muller transform.

This module holds no arithmetic of the min-cut method; it only produces
numbers that both the oracle and the GPU path consume as inputs.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_S30 = np.uint64(30)
_S27 = np.uint64(27)
_S31 = np.uint64(31)
_S11 = np.uint64(11)
_TWO_M53 = 2.0 ** -53


def _mix(z):
    """SplitMix64 step: add the golden-ratio increment, then finalise."""
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> _S30)) * _M1
        z = (z ^ (z >> _S27)) * _M2
        return z ^ (z >> _S31)


def _stream_base(seed, stream):
    s = _mix(np.asarray([seed], dtype=np.uint64))
    return _mix(s ^ np.uint64(stream))[0]


def bits64(seed, stream, index):
    """64 random bits for each entry of `index` (array-like of non-negative ints)."""
    idx = np.asarray(index, dtype=np.uint64)
    return _mix(_stream_base(seed, stream) ^ idx)


def uniform(seed, stream, index):
    """Uniform doubles in [0, 1) with 53 random bits each."""
    return (bits64(seed, stream, index) >> _S11).astype(np.float64) * _TWO_M53


def uniform_range(seed, stream, count, lo, hi, start=0):
    """`count` uniforms in [lo, hi) from indices start..start+count-1."""
    u = uniform(seed, stream, np.arange(start, start + count, dtype=np.uint64))
    return lo + (hi - lo) * u


def normal(seed, stream, count):
    """`count` standard normal variates by Box-Muller on consecutive pairs."""
    pairs = (count + 1) // 2
    j = np.arange(pairs, dtype=np.uint64)
    u1 = uniform(seed, stream, 2 * j)
    u2 = uniform(seed, stream, 2 * j + np.uint64(1))
    r = np.sqrt(-2.0 * np.log1p(-u1))          # 1-u1 lies in (0, 1]
    ang = 2.0 * np.pi * u2
    out = np.empty(2 * pairs, dtype=np.float64)
    out[0::2] = r * np.cos(ang)
    out[1::2] = r * np.sin(ang)
    return out[:count]
