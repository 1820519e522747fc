"""Ideal data volume of Section 4.3 (the read volume of Eq. 8 and the write
volume of Eq. 9).  Test and measurement infrastructure only.

Each term uses the width of the array it reads or writes: A's row pointers
for the first term, B's row pointers for the 4 s_rowPtr term, column and
value widths of B for the intermediate-product term, and C's widths for the
write volume.
"""


def ideal_volume(n_a, nnz_a, n_interprod, n_c, nnz_c, *, s_rp_a, s_rp_b, s_col_a, s_col_b,
                 s_val, s_rp_c, s_col_c):
    read = (2 * (n_a + 1) * s_rp_a
            + nnz_a * (4 * s_rp_b + 2 * s_col_a + s_val)
            + n_interprod * (2 * s_col_b + s_val))
    write = (n_c + 1) * s_rp_c + nnz_c * (s_col_c + s_val)
    return read, write
