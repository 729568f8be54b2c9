"""Canonical compressed layouts of the sampled set Phi (Sec. II.C, Eq. (5)).

The iterate Y of SVT is supported on Phi (Y^0 = c delta P_Phi(M), and every
update adds delta P_Phi(M - X)), so a sparse layout of Phi is fixed once per
solve.  This module defines, by plain sorting, what the device-side build
must produce bit for bit:

* CSR: entries sorted by (row, col); row_ptr[i] = number of entries in rows
  < i; col_idx the column of each entry; `order[e]` the position in the
  caller's input of CSR entry e.
* CSC: entries sorted by (col, row); col_ptr, row_idx likewise; perm[e] the
  CSR position of CSC entry e.

Inputs with an index out of range or a repeated cell are rejected.
"""

import numpy as np


class CSRError(ValueError):
    pass


def canonical_csr(m, n, rows, cols):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if rows.shape != cols.shape or rows.ndim != 1:
        raise CSRError("rows and cols must be 1-D arrays of equal length")
    if rows.size and (rows.min() < 0 or rows.max() >= m or cols.min() < 0
                      or cols.max() >= n):
        raise CSRError("index out of range")
    order = np.lexsort((cols, rows))            # primary key: row
    r_s, c_s = rows[order], cols[order]
    if rows.size > 1:
        dup = (r_s[1:] == r_s[:-1]) & (c_s[1:] == c_s[:-1])
        if dup.any():
            raise CSRError("duplicate cell")
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r_s, minlength=m), out=row_ptr[1:])
    perm = np.lexsort((r_s, c_s))               # CSR positions in CSC order
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(c_s, minlength=n), out=col_ptr[1:])
    return dict(row_ptr=row_ptr, col_idx=c_s, order=order,
                col_ptr=col_ptr, row_idx=r_s[perm], perm=perm)
