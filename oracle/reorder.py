"""Fine-level histogram, prefix sum and reorder of one row's products
(Section 3.2, Algorithm 3), as plain sequential loops.  Test infrastructure
only.

Given the column indices and values of a row's intermediate product, a chunk
length 2^shift and a base column, the chunk of a product is
(col - base) >> shift.  Products are counted per chunk, the counts are
scanned into offsets, and each product is written at offset[chunk] +
running count[chunk] with its column shifted into the chunk-local range.
Sequential reordering is a stable counting sort by chunk.
"""
import numpy as np


def reorder_row(cols, vals, shift: int, base: int, n_chunks: int):
    counts = [0] * n_chunks
    for c in cols:
        counts[(int(c) - base) >> shift] += 1
    offsets = [0] * (n_chunks + 1)
    for j in range(n_chunks):
        offsets[j + 1] = offsets[j] + counts[j]
    counts = [0] * n_chunks
    col_fine = np.zeros(len(cols), dtype=np.int64)
    val_fine = np.zeros(len(cols), dtype=np.float64)
    for c, v in zip(cols, vals):
        ch = (int(c) - base) >> shift
        pos = offsets[ch] + counts[ch]
        counts[ch] += 1
        col_fine[pos] = int(c) - base - (ch << shift)
        val_fine[pos] = float(v)
    return np.asarray(offsets, dtype=np.int64), col_fine, val_fine
