"""Block-sparse-row container used to hand Hamiltonians around.

Layout (the one the C ABI takes):
  row_ptr  int64 [n_block_rows + 1], monotone, row_ptr[0] == 0
  col_idx  int32 [nnzb], strictly increasing inside each block row
  values   float64 [nnzb, bd, bd], each block row-major
plus the spectral interval [e_min, e_max] that the input's construction
guarantees to contain the spectrum.
"""

from dataclasses import dataclass, field

import hashlib
import numpy as np


@dataclass
class BSR:
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray
    block_dim: int
    e_min: float
    e_max: float
    meta: dict = field(default_factory=dict)

    @property
    def n_block_rows(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def n(self) -> int:
        return self.n_block_rows * self.block_dim

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    def block_rows(self) -> np.ndarray:
        """Block-row index of every stored block (int64 [nnzb])."""
        return np.repeat(np.arange(self.n_block_rows, dtype=np.int64),
                         np.diff(self.row_ptr))

    def to_scipy(self):
        import scipy.sparse as sp
        bd = self.block_dim
        if bd == 1:
            return sp.csr_matrix((self.values.reshape(-1), self.col_idx, self.row_ptr),
                                 shape=(self.n, self.n))
        return sp.bsr_matrix((self.values, self.col_idx, self.row_ptr),
                             shape=(self.n, self.n), blocksize=(bd, bd))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    def digest(self) -> str:
        """sha256 over pattern and values, used to check that two machines built the same input."""
        h = hashlib.sha256()
        for a in (self.row_ptr, self.col_idx, self.values):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.array([self.e_min, self.e_max], dtype=np.float64).tobytes())
        return h.hexdigest()

    def with_values(self, values: np.ndarray) -> "BSR":
        return BSR(self.row_ptr, self.col_idx, np.ascontiguousarray(values, dtype=np.float64),
                   self.block_dim, self.e_min, self.e_max, dict(self.meta))
