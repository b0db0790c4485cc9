"""Plan object over the C ABI (argument marshalling only)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi as A


def _arr(x, dt):
    return np.ascontiguousarray(x, dtype=dt)


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class _BlockArgs:
    """Keeps the arrays of one hfx_blocks alive while the library reads them."""

    def __init__(self, b, data=None, on_device=False):
        self.row = _arr(b.row, np.int32)
        self.col = _arr(b.col, np.int32)
        self.R = _arr(b.R, np.int32).reshape(-1)
        self.off = _arr(b.off, np.int64)
        self.data_keep = None
        if data is None:
            data = b.data
        if on_device:
            self.data_ptr = int(data.data_ptr())
            self.data_keep = data
        elif data is None:
            self.data_ptr = None
        else:
            self.data_keep = _arr(data, np.float64)
            self.data_ptr = self.data_keep.ctypes.data
        self.s = A.Blocks(int(self.row.shape[0]), self.row.ctypes.data, self.col.ctypes.data, self.R.ctypes.data,
                          self.off.ctypes.data, self.data_ptr, 1 if on_device else 0)


class Plan:
    """Per-geometry plan (Algorithm 5, "Calculate C and V") for one or more cells.

    cells: objects with ``lattice`` (3,3), ``pos`` (n,3), ``species`` (n,), ``species_table`` [(n_ao, n_abf)]
    C, V, D_pattern: per-cell block sets with ``row``, ``col``, ``R``, ``off``, ``data`` (host numpy)
    thresholds: dict with eps_C, eps_V, eps_D, eps_cs_eri, eps_cs_mat
    """

    def __init__(self, cells, C, V, D_pattern, thresholds, precision=A.PREC_FP64, stages=A.SCREEN_ALL,
                 scheduler=A.SCHED_LPT, home_subset=None, stream=None, n_slots=0, max_device_bytes=0,
                 tier_tau=0.0, tier_tau_bf=0.0, mlp_weights=None, use_graph=False, tuning_db=None, tile_r=0):
        import torch
        self._torch = torch
        L = A.lib()
        self.n_cells = len(cells)
        self.n_basis = [int(sum(int(cl.species_table[int(t)][0]) for t in np.asarray(cl.species).reshape(-1)))
                        for cl in cells]
        self._keep = []
        ccells = (A.Cell * self.n_cells)()
        for i, cl in enumerate(cells):
            pos = _arr(cl.pos, np.float64).reshape(-1)
            sp = _arr(cl.species, np.int32)
            tab = (A.Species * len(cl.species_table))(*[A.Species(int(a), int(b)) for a, b in cl.species_table])
            self._keep += [pos, sp, tab]
            ccells[i].n_atoms = int(sp.shape[0])
            for k, v in enumerate(np.asarray(cl.lattice, np.float64).reshape(-1)):
                ccells[i].lattice[k] = float(v)
            ccells[i].pos = pos.ctypes.data
            ccells[i].species = sp.ctypes.data
            ccells[i].n_species = len(cl.species_table)
            ccells[i].sp = tab
        cargs = [_BlockArgs(b) for b in C]
        vargs = [_BlockArgs(b) for b in V]
        dargs = [_BlockArgs(b, data=np.zeros(0)) for b in D_pattern]
        cC = (A.Blocks * self.n_cells)(*[a.s for a in cargs])
        cV = (A.Blocks * self.n_cells)(*[a.s for a in vargs])
        cD = (A.Blocks * self.n_cells)(*[a.s for a in dargs])
        th = A.Thresholds(thresholds["eps_C"], thresholds["eps_V"], thresholds["eps_D"], thresholds["eps_cs_eri"],
                          thresholds["eps_cs_mat"])
        self.eps_mat = float(thresholds["eps_cs_mat"])
        hs = None if home_subset is None else _arr(home_subset, np.int32)
        if hs is not None and hs.shape[0] == 0:
            hs = np.zeros(1, np.int32)[:0]  # an empty subset still passes a non-NULL pointer
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        opt = A.Options(precision, stages, tier_tau, tier_tau_bf, scheduler,
                        None if mlp_weights is None else str(mlp_weights).encode(),
                        ctypes.c_void_p(stream.cuda_stream), None if hs is None else hs.ctypes.data,
                        0 if hs is None else int(hs.shape[0]), int(max_device_bytes), int(n_slots),
                        1 if use_graph else 0, None if tuning_db is None else str(tuning_db).encode(),
                        int(tile_r))
        h = ctypes.c_void_p()
        A.check(L.hfx_plan_create(self.n_cells, ctypes.byref(ccells), ctypes.byref(cC), ctypes.byref(cV),
                                  ctypes.byref(cD), ctypes.byref(th), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self.layouts = []
        self.sizes = []
        for c in range(self.n_cells):
            lay = A.Blocks()
            n = ctypes.c_int64()
            A.check(L.hfx_sigma_layout(h, c, ctypes.byref(lay), ctypes.byref(n)))
            nb = lay.n_blocks
            off = np.ctypeslib.as_array(ctypes.cast(lay.off, ctypes.POINTER(ctypes.c_int64)), shape=(nb + 1,)).copy()
            self.layouts.append(off)
            self.sizes.append(int(n.value))
        self.last_stats = None
        buf = ctypes.create_string_buffer(256)
        A.check(L.hfx_tune_key(h, buf, 256))
        self.tune_key = buf.value.decode()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                A.lib().hfx_plan_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    # ------------------------------------------------------------------ D marshalling
    def _d_struct(self, D):
        """D: per-cell block sets; data may be numpy (host) or a CUDA tensor (device)."""
        args = []
        for b in D:
            dev = hasattr(b.data, "data_ptr")
            args.append(_BlockArgs(b, on_device=dev))
        return args, (A.Blocks * self.n_cells)(*[a.s for a in args])

    def alloc_sigma(self):
        torch = self._torch
        return [torch.empty(n, dtype=torch.float64, device="cuda") for n in self.sizes]

    def build(self, D, sigma=None, stats=False):
        """Sigma^X on the D pattern of every cell (device float64 tensors, compact layout)."""
        args, cD = self._d_struct(D)
        if sigma is None:
            sigma = self.alloc_sigma()
        ptrs = (ctypes.c_void_p * self.n_cells)(*[s.data_ptr() for s in sigma])
        st = A.BuildStats() if stats else None
        A.check(A.lib().hfx_build(self._h, ctypes.byref(cD), ptrs, None if st is None else ctypes.byref(st)))
        self._last_args = args  # keep host/device inputs alive until the stream passes the build
        if st is not None:
            self.last_stats = st.as_dict()
        return sigma

    def energy(self, D, sigma):
        args, cD = self._d_struct(D)
        ptrs = (ctypes.c_void_p * self.n_cells)(*[s.data_ptr() for s in sigma])
        e = (ctypes.c_double * self.n_cells)()
        A.check(A.lib().hfx_energy(self._h, ctypes.byref(cD), ptrs, e))
        del args
        return list(e)

    def sigma_to_k(self, sigma, kfrac, cell=0, out=None):
        """H(k) = sum_R exp(i 2 pi k.R) Sigma(R) of one cell at the k-points ``kfrac`` ([n_k, 3],
        fractional): a device complex128 tensor [n_k, n_basis, n_basis] (``out`` if given).
        ``sigma``: the cell's device Sigma (or the list hfx_build returned).  Stream-ordered."""
        torch = self._torch
        if isinstance(sigma, (list, tuple)):
            sigma = sigma[cell]
        k = np.ascontiguousarray(np.asarray(kfrac, np.float64).reshape(-1, 3))
        if not 0 <= cell < self.n_cells:
            # rejected by the library (HFX_ERR_ARG) before it touches any array
            A.check(A.lib().hfx_sigma_to_k(self._h, int(cell), None, int(k.shape[0]), _ptr(k), None))
        nb = self.n_basis[cell]
        if out is None:
            out = torch.empty((k.shape[0], nb, nb), dtype=torch.complex128, device="cuda")
        if out.dtype != torch.complex128 or tuple(out.shape) != (k.shape[0], nb, nb) or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous complex128 tensor of shape {(k.shape[0], nb, nb)}")
        if sigma.dtype != torch.float64 or not sigma.is_cuda or sigma.numel() != self.sizes[cell]:
            raise ValueError(f"sigma must be the cell's device float64 Sigma ({self.sizes[cell]} elements)")
        A.check(A.lib().hfx_sigma_to_k(self._h, int(cell), ctypes.c_void_p(sigma.data_ptr()), int(k.shape[0]),
                                       _ptr(k), ctypes.c_void_p(out.data_ptr())))
        return out

    def density_from_k(self, ck, occ, kfrac, cell=0, out=None):
        """D(R) on the cell's D pattern (device float64, hfx_sigma_layout order) from eigenvectors
        ``ck`` (device complex128 [n_k, n_basis, n_occ]) and occupations ``occ`` (device float64
        [n_k, n_occ]) at the k-points ``kfrac`` ([n_k, 3], fractional).  Stream-ordered."""
        torch = self._torch
        k = np.ascontiguousarray(np.asarray(kfrac, np.float64).reshape(-1, 3))
        if not 0 <= cell < self.n_cells:
            A.check(A.lib().hfx_density_from_k(self._h, int(cell), int(k.shape[0]), _ptr(k), 0, None, None, None))
        nb = self.n_basis[cell]
        n_occ = int(ck.shape[2]) if ck.dim() == 3 else -1
        if (ck.dtype != torch.complex128 or not ck.is_cuda or not ck.is_contiguous()
                or tuple(ck.shape) != (k.shape[0], nb, n_occ)):
            raise ValueError(f"ck must be a contiguous device complex128 tensor [{k.shape[0]}, {nb}, n_occ]")
        if occ.dtype != torch.float64 or not occ.is_cuda or not occ.is_contiguous() \
                or tuple(occ.shape) != (k.shape[0], n_occ):
            raise ValueError(f"occ must be a contiguous device float64 tensor [{k.shape[0]}, {n_occ}]")
        if out is None:
            out = torch.empty(self.sizes[cell], dtype=torch.float64, device="cuda")
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() != self.sizes[cell]:
            raise ValueError(f"out must be a device float64 tensor of {self.sizes[cell]} elements")
        A.check(A.lib().hfx_density_from_k(self._h, int(cell), int(k.shape[0]), _ptr(k), n_occ,
                                           ctypes.c_void_p(ck.data_ptr()), ctypes.c_void_p(occ.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr())))
        return out

    def item_features(self, mu, sd):
        """Scheduler features of every item from the last build (device float32 tensor
        [n_items, ITEM_FEATURES])."""
        torch = self._torch
        mu = np.ascontiguousarray(mu, np.float32)
        sd = np.ascontiguousarray(sd, np.float32)
        if mu.shape != (A.ITEM_FEATURES,) or sd.shape != (A.ITEM_FEATURES,):
            raise ValueError(f"mu and sd must hold {A.ITEM_FEATURES} values")
        n = ctypes.c_int64()
        A.check(A.lib().hfx_item_profile(self._h, ctypes.byref(n), None, None, None))
        X = torch.empty((n.value, A.ITEM_FEATURES), dtype=torch.float32, device="cuda")
        A.check(A.lib().hfx_item_features(self._h, _ptr(mu), _ptr(sd), ctypes.c_void_p(X.data_ptr())))
        return X

    def item_profile(self):
        """Per-item labels of the last build: (ticks, kept-unit counters [n, 5], contribution bound)."""
        n = ctypes.c_int64()
        A.check(A.lib().hfx_item_profile(self._h, ctypes.byref(n), None, None, None))
        cyc = np.zeros(n.value, np.int64)
        units = np.zeros((n.value, A.ITEM_UNITS), np.int64)
        contrib = np.zeros(n.value, np.float64)
        A.check(A.lib().hfx_item_profile(self._h, ctypes.byref(n), _ptr(cyc), _ptr(units), _ptr(contrib)))
        return cyc, units, contrib
