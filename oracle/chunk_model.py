"""Chunk-count model of Section 3.5 (Eqs. 2-7), written out as printed.
Test infrastructure only (see the package docstring).

Symbols follow the paper: m_C columns of C (ceiled to a power of two),
s_L2 the cache the fine-level structures must fit, s_cacheLine, and
s_denseAccum = s_val + 1 for the numeric phase (a value plus one bitmap byte)
or 1 for the symbolic phase.  The per-chunk reorder storage is
s_chunkFine = s_histoType + s_prefixSumType + 2 s_cacheLine with four-byte
histogram and prefix types.
"""
from __future__ import annotations

import math


def pow2_ceil(x: float) -> int:
    """Smallest power of two >= x (x >= 1)."""
    p = 1
    while p < x:
        p <<= 1
    return p


def pow2_floor(x: float) -> int:
    """Largest power of two <= x (x >= 1)."""
    if x < 1:
        raise ValueError("x must be >= 1")
    p = 1
    while p * 2 <= x:
        p <<= 1
    return p


def pow2_nearest(x: float) -> int:
    """Power of two nearest to x in log2 (ties go up).  The paper says
    'rounded to the nearest power of two' without naming the scale; log2 is
    the reading taken here."""
    if x <= 1:
        return 1
    e = math.log2(x)
    lo = math.floor(e)
    return 1 << (lo + 1 if e - lo >= 0.5 else lo)


def s_chunk_fine(s_cache_line: int, s_histo: int = 4, s_prefix: int = 4) -> int:
    return s_histo + s_prefix + 2 * s_cache_line


def fine_storage(m_c: int, n_chunks: int, s_dense_accum: float, s_chunk: float) -> float:
    """Eq. 2: storage of the cached fine-level structures."""
    return m_c * s_dense_accum / n_chunks + n_chunks * s_chunk


def paper_fine_nchunks(m_c: int, s_dense_accum: float, s_chunk: float) -> int:
    """Eq. 3 (and Eq. 6 with m_C = m_CmaxL2): the minimiser of Eq. 2,
    rounded to the nearest power of two."""
    return pow2_nearest(math.sqrt(m_c * s_dense_accum / s_chunk))


def fine_storage_opt(m_c: int, s_dense_accum: float, s_chunk: float) -> float:
    """Eq. 4: Eq. 2 at the unrounded optimum."""
    return 2.0 * math.sqrt(m_c * s_dense_accum * s_chunk)


def paper_mcmax(s_l2: int, s_dense_accum: float, s_chunk: float) -> int:
    """Eq. 5: largest m_C whose optimal fine-level storage fits s_L2,
    floored to a power of two."""
    return pow2_floor(s_l2 * s_l2 / (4.0 * s_dense_accum * s_chunk))


def paper_model(m_c: int, s_l2: int, s_cache_line: int, s_val: int, phase: str = "numeric"):
    """Eqs. 2-7 for one matrix: the fine chunk count alone when the fine-level
    structures fit s_L2 (strictly), else the two-level split."""
    m_c = pow2_ceil(max(1, m_c))
    sd = (s_val + 1) if phase == "numeric" else 1
    sc = s_chunk_fine(s_cache_line)
    mcmax = paper_mcmax(s_l2, sd, sc)
    fits = fine_storage_opt(m_c, sd, sc) < s_l2
    if fits:
        nf = min(paper_fine_nchunks(m_c, sd, sc), m_c)
        return {"m_c": m_c, "use_coarse": False, "n_chunks_fine": nf, "n_chunks_coarse": 1,
                "chunk_len_fine": m_c // nf, "chunk_len_coarse": m_c, "m_cmax": mcmax}
    nf = min(paper_fine_nchunks(mcmax, sd, sc), mcmax)
    nco = max(1, m_c // mcmax)  # Eq. 7
    return {"m_c": m_c, "use_coarse": True, "n_chunks_fine": nf, "n_chunks_coarse": nco,
            "chunk_len_fine": mcmax // nf, "chunk_len_coarse": m_c // nco, "m_cmax": mcmax}
