"""ctypes binding of librfo.so (argument marshalling only).

Each method of Engine forwards to the C entry point of the same name declared in
include/rfo.h; all arithmetic runs in the library's HIP kernels.  PyTorch is
imported first so that the library binds to the HIP runtime PyTorch loaded, and
torch tensors (host or device) can be passed wherever the ABI takes a pointer.
"""

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library will share)

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librfo.so")

RFO_OK = 0
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x2": 3}
STATUS = {0: "RFO_OK", -1: "RFO_E_INVALID", -2: "RFO_E_STATE", -3: "RFO_E_NOMEM",
          -4: "RFO_E_DEVICE", -5: "RFO_E_NUMERIC", -6: "RFO_E_UNSUPPORTED"}

_lib = None


class RfoError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{STATUS.get(code, code)}: {message}")
        self.code = code
        self.status = STATUS.get(code, str(code))


def library_path() -> str:
    return _LIB_PATH


def load():
    """Loads librfo.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with python -m paper_1812_05264_amd.build")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.rfo_create.argtypes = [ctypes.POINTER(vp), i32, vp]
    lib.rfo_destroy.argtypes = [vp]
    lib.rfo_destroy.restype = None
    lib.rfo_last_error.argtypes = [vp]
    lib.rfo_last_error.restype = ctypes.c_char_p
    lib.rfo_set_hamiltonian.argtypes = [vp, i64, i32, vp, vp, vp, dbl, dbl, i32]
    lib.rfo_get_interval.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.rfo_set_probes.argtypes = [vp, i64, vp, vp]
    lib.rfo_fermi_moments.argtypes = [vp, dbl, dbl, i64, vp, vp, vp]
    lib.rfo_energy_and_dEdH.argtypes = [vp, dbl, dbl, i64, vp, vp]
    lib.rfo_fermi_moments_noalloc.argtypes = [vp, dbl, dbl, i64, vp, vp]
    lib.rfo_hf_forces.argtypes = [vp, vp, vp]
    lib.rfo_hf_forces_overlap.argtypes = [vp, vp, vp, vp]
    lib.rfo_get_dFdS.argtypes = [vp, vp]
    lib.rfo_set_timing.argtypes = [vp, i32]
    lib.rfo_set_moment_doubling.argtypes = [vp, i32]
    lib.rfo_set_tuning.argtypes = [vp, i32, i64]
    lib.rfo_traces_at.argtypes = [vp, dbl, dbl, ctypes.POINTER(dbl)]
    lib.rfo_set_overlap.argtypes = [vp, vp, dbl]
    lib.rfo_get_density_q.argtypes = [vp, vp]
    lib.rfo_density_forces.argtypes = [vp, vp, vp, vp]
    lib.rfo_cg_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.rfo_step_timing.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.rfo_rational_fit.argtypes = [i32, dbl, dbl, dbl, dbl, vp, vp, vp, vp]
    lib.rfo_rational_estimate.argtypes = [vp, dbl, i64, vp, vp, vp, vp, dbl, i64, vp, vp, vp, vp]
    lib.rfo_rational_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.rfo_color_atoms.argtypes = [i64, vp, dbl, vp, ctypes.POINTER(i32)]
    lib.rfo_set_colored_probes.argtypes = [vp, vp, i32, vp]
    for f in (
        "rfo_create", "rfo_set_hamiltonian", "rfo_get_interval", "rfo_set_probes",
        "rfo_fermi_moments", "rfo_fermi_moments_noalloc", "rfo_energy_and_dEdH", "rfo_hf_forces",
        "rfo_set_timing", "rfo_step_timing", "rfo_set_moment_doubling", "rfo_set_tuning",
        "rfo_traces_at", "rfo_set_overlap", "rfo_get_density_q", "rfo_density_forces",
        "rfo_cg_stats", "rfo_rational_fit", "rfo_rational_estimate", "rfo_rational_stats", "rfo_color_atoms",
        "rfo_set_colored_probes", "rfo_hf_forces_overlap", "rfo_get_dFdS"):
        getattr(lib, f).restype = i32
    _lib = lib
    return lib


def _ptr(a):
    """Address of a contiguous numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return a.ctypes.data


def _host(a, dtype):
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


def _numel(a):
    return a.numel() if isinstance(a, torch.Tensor) else int(np.asarray(a).size)


def _need(a, n, what):
    """The C ABI takes plain pointers: a buffer of the wrong size would be read or
    written past its end, so every size is checked here.  n = 0 (no Hamiltonian
    yet) checks nothing: the library then rejects the call by its state."""
    if a is not None and n > 0 and _numel(a) != n:
        raise ValueError(f"{what} must hold {n} values (got {_numel(a)})")


def _out_f64(a, n, what):
    """A caller-supplied output buffer: FP64, contiguous, n values (None passes)."""
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64:
            raise TypeError(f"{what} must be float64")
    elif np.asarray(a).dtype != np.float64:
        raise TypeError(f"{what} must be float64")
    _need(a, n, what)
    return a


def _in_f64(a, n, what):
    """An input block array: torch tensors stay where they are (FP64, made
    contiguous), anything else becomes a contiguous FP64 host array; n values."""
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64:
            raise TypeError(f"{what} must be float64")
        a = a.contiguous()
    else:
        a = np.ascontiguousarray(a, dtype=np.float64)
    _need(a, n, what)
    return a


def _complex_pairs(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1))


def color_atoms(positions, r_max):
    """Welsh-Powell colours [N] (int64) of the atoms for the multi-color probe ensemble
    (rfo_color_atoms, host-only)."""
    lib = load()
    pos = np.ascontiguousarray(positions, dtype=np.float64)
    if pos.ndim != 2 or pos.shape[1] != 3:
        raise ValueError("positions must be [N, 3]")
    out = np.empty(pos.shape[0], dtype=np.int32)
    q = ctypes.c_int32()
    rc = lib.rfo_color_atoms(pos.shape[0], _ptr(pos), float(r_max), _ptr(out), ctypes.byref(q))
    if rc != 0:
        raise RfoError(rc, "rfo_color_atoms failed")
    return out.astype(np.int64)


def rational_fit(n_nodes, T, mu, e_min, e_max):
    """Pole fit of f and g (rfo_rational_fit, host only): dict(poles, res_f, res_g
    (complex arrays of 2 n_nodes), f0, g0, g1)."""
    lib = load()
    m = 2 * int(n_nodes)
    z, wf, wg = (np.empty((m, 2)) for _ in range(3))
    poly = np.empty(3)
    rc = lib.rfo_rational_fit(int(n_nodes), float(T), float(mu), float(e_min), float(e_max),
                              _ptr(z), _ptr(wf), _ptr(wg), _ptr(poly))
    if rc != RFO_OK:
        raise RfoError(rc, "rfo_rational_fit rejected its arguments")
    cx = lambda a: a[:, 0] + 1j * a[:, 1]
    return {"poles": cx(z), "res_f": cx(wf), "res_g": cx(wg), "f0": float(poly[0]),
            "g0": float(poly[1]), "g1": float(poly[2])}


class Engine:
    """One library context on one GPU, issuing work on one HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = load()
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream(device)
        handle = stream.cuda_stream if isinstance(stream, torch.cuda.Stream) else stream
        ctx = ctypes.c_void_p()
        rc = self._lib.rfo_create(ctypes.byref(ctx), int(device), handle)
        if rc != RFO_OK:
            raise RfoError(rc, self._lib.rfo_last_error(None).decode())
        self._ctx = ctx
        self.device = device
        self.n_block_rows = 0
        self.block_dim = 0
        self.nnzb = 0
        self.n_probes = 0
        self.precision = "fp64"

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.rfo_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != RFO_OK:
            raise RfoError(rc, self._lib.rfo_last_error(self._ctx).decode())

    # -- rfo_set_hamiltonian ------------------------------------------------------
    def set_hamiltonian(self, row_ptr, col_idx, values, block_dim, e_min=0.0, e_max=0.0,
                        precision="fp64"):
        """row_ptr/col_idx: host arrays (None, None keeps the pattern); values: FP64
        [nnzb, bd, bd] numpy array or torch tensor (host or device).  e_min >= e_max
        asks for the widened Gershgorin interval."""
        bd = int(block_dim)
        if row_ptr is None and col_idx is None:
            rp = ci = None
            nb = self.n_block_rows
            nnzb = self.nnzb
        else:
            rp = _host(row_ptr, np.int64).ravel()
            ci = _host(col_idx, np.int32).ravel()
            if rp.shape[0] < 2:
                raise ValueError("row_ptr must hold n_block_rows + 1 >= 2 entries")
            nb = rp.shape[0] - 1
            nnzb = int(rp[-1])
            _need(ci, nnzb, "col_idx")
        # other block sizes are rejected by the library before it reads the values
        vals = _in_f64(values, nnzb * bd * bd if bd in (1, 9) else 0, "values")
        self._keep = (rp, ci, vals)
        self._check(self._lib.rfo_set_hamiltonian(self._ctx, nb, int(block_dim), _ptr(rp), _ptr(ci),
                                                  _ptr(vals), float(e_min), float(e_max),
                                                  PRECISIONS[precision]))
        self._keep = None
        self.n_block_rows = nb
        self.block_dim = bd
        self.nnzb = nnzb
        self.precision = precision
        return self.interval()

    def set_values(self, values):
        """Replaces the values, keeping pattern, interval and precision."""
        a, b = self.interval()
        return self.set_hamiltonian(None, None, values, self.block_dim, a, b, self.precision)

    def interval(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.rfo_get_interval(self._ctx, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # -- rfo_set_probes -------------------------------------------------------------
    def set_probes(self, R, weights=None):
        """R [n, s] (n = n_block_rows * block_dim rows, s probes); weights [s] or None."""
        R = _host(R, np.float64)
        n = self.n_block_rows * self.block_dim
        if R.ndim != 2 or (n > 0 and R.shape[0] != n):
            raise ValueError(f"R must be [{n}, s] (got {list(R.shape)})")
        w = None if weights is None else _host(weights, np.float64)
        _need(w, R.shape[1], "weights")
        self._check(self._lib.rfo_set_probes(self._ctx, int(R.shape[1]), _ptr(R), _ptr(w)))
        self.n_probes = int(R.shape[1])

    def set_colored_probes(self, colours, n_orb, signs):
        """One sample of the multi-color ensemble, built by the library (weights one)."""
        col = np.ascontiguousarray(colours, dtype=np.int32)
        sg = np.ascontiguousarray(signs, dtype=np.float64)
        n = self.n_block_rows * self.block_dim
        if n > 0 and (int(n_orb) < 1 or n % int(n_orb) != 0):
            raise ValueError(f"n_orb must divide the {n} rows")
        _need(col, n // int(n_orb) if n > 0 else 0, "colours")
        _need(sg, n, "signs")
        self._check(self._lib.rfo_set_colored_probes(self._ctx, _ptr(col), int(n_orb), _ptr(sg)))
        self.n_probes = (int(col.max()) + 1) * int(n_orb)

    # -- rfo_fermi_moments ----------------------------------------------------------
    def fermi_moments(self, T, mu, n_terms, moments=True, density=False, density_out=None):
        """Returns dict(N, E, F, moments [s, p] or None, density [nnzb, bd, bd] or None).
        density_out may be a preallocated FP64 torch tensor (host or device)."""
        mom = np.empty((self.n_probes, int(n_terms))) if moments else None
        nef = np.empty(3)
        dens = _out_f64(density_out, self.nnzb * self.block_dim * self.block_dim, "density_out")
        if density and dens is None:
            dens = np.empty((self.nnzb, self.block_dim, self.block_dim))
        self._check(self._lib.rfo_fermi_moments(self._ctx, float(T), float(mu), int(n_terms),
                                                _ptr(mom), _ptr(nef), _ptr(dens)))
        return {"N": float(nef[0]), "E": float(nef[1]), "F": float(nef[2]), "moments": mom,
                "density": dens}

    # -- rfo_fermi_moments_noalloc --------------------------------------------------
    def fermi_moments_noalloc(self, T, mu, n_terms, moments=True):
        """The moment-only call without device allocation (library scratch array).
        Returns dict(N, E, F, moments [s, p] or None)."""
        mom = np.empty((self.n_probes, int(n_terms))) if moments else None
        nef = np.empty(3)
        self._check(self._lib.rfo_fermi_moments_noalloc(self._ctx, float(T), float(mu), int(n_terms),
                                                        _ptr(mom), _ptr(nef)))
        return {"N": float(nef[0]), "E": float(nef[1]), "F": float(nef[2]), "moments": mom}

    # -- rfo_energy_and_dEdH --------------------------------------------------------
    def energy_and_dEdH(self, T, mu, n_terms, gradient=True, dFdH_out=None):
        nef = np.empty(3)
        g = _out_f64(dFdH_out, self.nnzb * self.block_dim * self.block_dim, "dFdH_out")
        if gradient and g is None:
            g = np.empty((self.nnzb, self.block_dim, self.block_dim))
        self._check(self._lib.rfo_energy_and_dEdH(self._ctx, float(T), float(mu), int(n_terms),
                                                  _ptr(nef), _ptr(g)))
        return {"N": float(nef[0]), "E": float(nef[1]), "F": float(nef[2]), "dFdH": g}

    # -- rfo_hf_forces --------------------------------------------------------------
    def hf_forces(self, dHdR):
        """dHdR [nnzb, 3, bd, bd] (host or device FP64): forces [n_block_rows, 3]."""
        d = _in_f64(dHdR, self.nnzb * 3 * self.block_dim * self.block_dim, "dHdR")
        out = np.empty((self.n_block_rows, 3))
        self._check(self._lib.rfo_hf_forces(self._ctx, _ptr(d), _ptr(out)))
        return out

    def hf_forces_overlap(self, dHdR, dSdR):
        """-(sum <dF/dH, dH/dR_a> + sum <dF/dS, dS/dR_a>) from the last gradient with an
        overlap, [n_block_rows, 3]."""
        nd = self.nnzb * 3 * self.block_dim * self.block_dim
        dH = _host(dHdR, np.float64)
        dS = None if dSdR is None else _host(dSdR, np.float64)
        _need(dH, nd, "dHdR")
        _need(dS, nd, "dSdR")
        out = np.empty((self.n_block_rows, 3))
        self._check(self._lib.rfo_hf_forces_overlap(self._ctx, _ptr(dH), _ptr(dS), _ptr(out)))
        return out

    def dFdS(self):
        """dF/dS blocks (symmetric part) of the last gradient with an overlap."""
        out = np.empty((self.nnzb, self.block_dim, self.block_dim))
        self._check(self._lib.rfo_get_dFdS(self._ctx, _ptr(out)))
        return out

    # -- instrumentation --------------------------------------------------------------
    def set_overlap(self, S_values=None, cg_tol=1e-13):
        """Overlap S [nnzb, bd, bd] on H's pattern (None: S = I)."""
        S = None if S_values is None else _host(S_values, np.float64)
        _need(S, self.nnzb * self.block_dim * self.block_dim, "S_values")
        self._check(self._lib.rfo_set_overlap(self._ctx, _ptr(S), float(cg_tol)))

    def density_q(self):
        """Q blocks of the last fermi_moments call with density and an overlap."""
        out = np.empty((self.nnzb, self.block_dim, self.block_dim))
        self._check(self._lib.rfo_get_density_q(self._ctx, _ptr(out)))
        return out

    def density_forces(self, dHdR, dSdR=None):
        """-(tr[P dH/dR_a] - tr[Q dS/dR_a]) from the last density blocks, [n_block_rows, 3]."""
        nd = self.nnzb * 3 * self.block_dim * self.block_dim
        dH = _host(dHdR, np.float64)
        dS = None if dSdR is None else _host(dSdR, np.float64)
        _need(dH, nd, "dHdR")
        _need(dS, nd, "dSdR")
        out = np.empty((self.n_block_rows, 3))
        self._check(self._lib.rfo_density_forces(self._ctx, _ptr(dH), _ptr(dS), _ptr(out)))
        return out

    # -- rfo_rational_estimate ------------------------------------------------------
    def rational(self, mu, fit, tol=1e-10, max_iter=100000, density=False, gradient=False,
                 density_out=None, dFdH_out=None):
        """Rational estimate with the fit dict of rational_fit (or any poles/residues of
        the same form).  Returns dict(N, E, F, density, dFdH, iterations).  With an
        overlap set the shifted systems are (H - z S) g = r, density_q() then holds the
        Q blocks of the call; the gradient with an overlap (requested without density) also
        leaves dF/dS for dFdS() and hf_forces_overlap()."""
        z, wf, wg = (_complex_pairs(fit[k]) for k in ("poles", "res_f", "res_g"))
        poly = np.array([fit["f0"], fit["g0"], fit["g1"]], dtype=np.float64)
        npol = z.shape[0]
        nef = np.empty(3)
        its = np.empty(npol, dtype=np.int64)
        nv = self.nnzb * self.block_dim * self.block_dim
        dens = _out_f64(density_out, nv, "density_out")
        if density and dens is None:
            dens = np.empty((self.nnzb, self.block_dim, self.block_dim))
        g = _out_f64(dFdH_out, nv, "dFdH_out")
        if gradient and g is None:
            g = np.empty((self.nnzb, self.block_dim, self.block_dim))
        self._check(self._lib.rfo_rational_estimate(
            self._ctx, float(mu), npol, _ptr(z), _ptr(wf), _ptr(wg), _ptr(poly), float(tol),
            int(max_iter), _ptr(nef), _ptr(dens), _ptr(g), _ptr(its)))
        return {"N": float(nef[0]), "E": float(nef[1]), "F": float(nef[2]), "density": dens,
                "dFdH": g, "iterations": its}

    def rational_stats(self):
        it, so = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.rfo_rational_stats(self._ctx, ctypes.byref(it), ctypes.byref(so)))
        return it.value, so.value

    def cg_stats(self):
        it, so = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.rfo_cg_stats(self._ctx, ctypes.byref(it), ctypes.byref(so)))
        return it.value, so.value

    def traces_at(self, T, mu):
        """N, E, F at (T, mu) from the moments of the last fermi_moments / energy call."""
        out = (ctypes.c_double * 3)()
        self._check(self._lib.rfo_traces_at(self._ctx, float(T), float(mu), out))
        return {"N": out[0], "E": out[1], "F": out[2]}

    def set_moment_doubling(self, enabled=True):
        """Moment-only fermi_moments calls run floor(p/2) steps (doubling identities)."""
        self._check(self._lib.rfo_set_moment_doubling(self._ctx, 1 if enabled else 0))

    TUNING = {"ppl": 0, "rpi": 1, "rows_per_wg": 2, "grid": 3, "bf16_chunks": 4, "sddmm_ppl": 5,
              "sddmm_mfma": 6, "sddmm_steps": 7, "sddmm_steps_bf16": 8, "overlap": 9,
              "cplx_ppl": 10, "cplx_rows": 11, "cplx_grid": 12, "adjoint_bytes": 13, "alt_sweep": 14,
              "adjoint_tail": 15}

    def set_tuning(self, key, value=-1):
        """Launch geometry / schedule of this context (rfo_set_tuning); -1 restores the default."""
        self._check(self._lib.rfo_set_tuning(self._ctx, self.TUNING[key], int(value)))

    def set_timing(self, enabled=True):
        self._check(self._lib.rfo_set_timing(self._ctx, 1 if enabled else 0))

    def step_timing(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self._lib.rfo_step_timing(self._ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
