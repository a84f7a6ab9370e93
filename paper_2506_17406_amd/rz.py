"""Thin ctypes binding of librz.so (the C ABI declared in include/rz.h).

Argument marshalling only: every step of setup, apply_A, apply_P and the PCG
solve runs inside the HIP library.  Device vectors are torch float64 tensors
on the GPU; their pointers and the current HIP stream are passed through.
Importing this module fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RZ_LIBRARY names another build of the same library (the host-sanitizer
# build of the CPU tests); by default the in-tree librz.so
LIB_PATH = os.environ.get("RZ_LIBRARY") or os.path.join(_HERE, "librz.so")

RZ_HGRAD, RZ_HCURL, RZ_HDIV, RZ_HCURL2, RZ_HDIV2 = 0, 1, 2, 3, 4
SPACES = {"CG": RZ_HGRAD, "hgrad": RZ_HGRAD, "Ned": RZ_HCURL, "hcurl": RZ_HCURL, "RT": RZ_HDIV, "hdiv": RZ_HDIV,
          "NedTwo": RZ_HCURL2, "hcurl2": RZ_HCURL2, "BDM": RZ_HDIV2, "hdiv2": RZ_HDIV2}
ERRORS = {0: "RZ_OK", -1: "RZ_ERR_ARG", -2: "RZ_ERR_UNSUPPORTED", -3: "RZ_ERR_MESH", -4: "RZ_ERR_DEGENERATE_CELL",
          -5: "RZ_ERR_NOT_SPD", -6: "RZ_ERR_NO_CONVERGENCE", -7: "RZ_ERR_BREAKDOWN", -8: "RZ_ERR_DEVICE",
          -9: "RZ_ERR_OOM"}


class RzMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_vertices", ctypes.c_int64), ("coords", ctypes.POINTER(ctypes.c_double)),
                ("n_cells", ctypes.c_int64), ("cells", ctypes.POINTER(ctypes.c_int64))]


RZ_FP64, RZ_FP32_IR, RZ_FP32_PC, RZ_BF16_PC = 0, 1, 2, 3
PRECISIONS = {"fp64": RZ_FP64, "fp32-ir": RZ_FP32_IR, "fp32-pc": RZ_FP32_PC, "bf16-pc": RZ_BF16_PC}
RZ_PC_ADDITIVE, RZ_PC_HYBRID = 0, 1
PCS = {"additive": RZ_PC_ADDITIVE, "hybrid": RZ_PC_HYBRID}
RZ_DECOMP_PAPER, RZ_DECOMP_VERTEX, RZ_DECOMP_VERTEX_FULL = 0, 1, 2
RZ_DECOMP_PAPER_FULL, RZ_DECOMP_HIPTMAIR, RZ_DECOMP_HIPTMAIR_FULL = 3, 4, 5
RZ_DECOMP_TYPEI, RZ_DECOMP_TYPEI_FULL = 6, 7
DECOMPOSITIONS = {"paper": RZ_DECOMP_PAPER, "vertex": RZ_DECOMP_VERTEX, "vertex-full": RZ_DECOMP_VERTEX_FULL,
                  "paper-full": RZ_DECOMP_PAPER_FULL, "hiptmair": RZ_DECOMP_HIPTMAIR,
                  "hiptmair-full": RZ_DECOMP_HIPTMAIR_FULL, "typeI": RZ_DECOMP_TYPEI,
                  "typeI-full": RZ_DECOMP_TYPEI_FULL}


class RzOptions(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_rtol", ctypes.c_double), ("pc", ctypes.c_int32),
                ("eager", ctypes.c_int32), ("decomposition", ctypes.c_int32),
                ("dirichlet_facet", ctypes.POINTER(ctypes.c_uint8)), ("coarse", ctypes.c_int32),
                ("mg_levels", ctypes.c_int32), ("mg_meshes", ctypes.POINTER(RzMesh))]


RZ_COARSE_EXACT, RZ_COARSE_MG = 0, 1
COARSE = {"exact": RZ_COARSE_EXACT, "mg": RZ_COARSE_MG}


class RzInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("cond_estimate", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("outer_iterations", ctypes.c_int32), ("setup_ms", ctypes.c_double)]


class RzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (python -m paper_2506_17406_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pi32, pi64, pdbl = ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(dbl)
    sig = {
        "rz_setup": (ctypes.c_int, [ctypes.POINTER(RzMesh), i32, ctypes.c_int, ctypes.POINTER(RzOptions), P,
                                    ctypes.POINTER(P)]),
        "rz_sizes": (ctypes.c_int, [P, pi64, pi64, pi32, pi32]),
        "rz_apply_A": (ctypes.c_int, [P, P, P, i32, i64, P]),
        "rz_apply_P": (ctypes.c_int, [P, P, P, i32, i64, P]),
        "rz_apply_A_fp32": (ctypes.c_int, [P, P, P, i32, i64, P]),
        "rz_apply_P_fp32": (ctypes.c_int, [P, P, P, i32, i64, P]),
        "rz_apply_A_noalloc": (ctypes.c_int, [P, P, P, i32, i64, P]),
        "rz_solve": (ctypes.c_int, [P, P, P, i32, i64, dbl, ctypes.POINTER(RzInfo), P]),
        "rz_pc_weights": (ctypes.c_int, [P, pdbl]),
        "rz_dirichlet_dofs": (ctypes.c_int, [P, pi64, pi32]),
        "rz_patch_set_info": (ctypes.c_int, [P, i32, pi32, pi64, pi32, pi64, pi64, pi64]),
        "rz_patch_set_apply": (ctypes.c_int, [P, i32, P, P, i32, i64, P]),
        "rz_export_topology": (ctypes.c_int, [P, pi32, pi64, pi64, pi64, pi32]),
        "rz_export_reference": (ctypes.c_int, [P, pdbl]),
        "rz_reference": (ctypes.c_int, [i32, i32, ctypes.c_int, pi32, pi32, pdbl]),
        "rz_numbering": (ctypes.c_int, [ctypes.POINTER(RzMesh), i32, ctypes.c_int, pi64, pi32, pi64, pi64, pi64,
                                        pi32]),
        "rz_patch_lists": (ctypes.c_int, [ctypes.POINTER(RzMesh), i32, ctypes.c_int, i32, pi64, pi64, pi64, pi32]),
        "rz_destroy": (None, [P]),
        "rz_set_apply_tiles": (ctypes.c_int, [P, i32, i32]),
        "rz_get_apply_tiles": (ctypes.c_int, [P, pi32]),
        "rz_batch_create": (ctypes.c_int, [ctypes.POINTER(P), i32, ctypes.POINTER(P)]),
        "rz_batch_solve": (ctypes.c_int, [P, ctypes.POINTER(P), ctypes.POINTER(P), dbl, ctypes.POINTER(RzInfo), P]),
        "rz_batch_destroy": (None, [P]),
        "rz_last_error": (ctypes.c_char_p, []),
        "rz_hodge_setup": (ctypes.c_int, [ctypes.POINTER(RzMesh), i32, i32, dbl, ctypes.POINTER(RzOptions), P,
                                          ctypes.POINTER(P)]),
        "rz_hodge_sizes": (ctypes.c_int, [P, pi64, pi64]),
        "rz_hodge_apply": (ctypes.c_int, [P, P, P, P]),
        "rz_hodge_apply_P": (ctypes.c_int, [P, P, P, P]),
        "rz_hodge_solve": (ctypes.c_int, [P, P, P, dbl, ctypes.POINTER(RzInfo), P]),
        "rz_hodge_destroy": (None, [P]),
        "rz_derivative_reference": (ctypes.c_int, [i32, i32, pi32, pi32, pdbl]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(code):
    if code != 0:
        raise RzError(code, lib.rz_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _mesh(coords, cells):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    m = RzMesh(coords.shape[1], coords.shape[0], _ptr(coords, ctypes.c_double), cells.shape[0],
               _ptr(cells, ctypes.c_int64))
    return m, (coords, cells)


def reference(dim, degree, space):
    """Stacked reference matrices (Q, n_loc, n_loc), host only."""
    n, Q = ctypes.c_int32(), ctypes.c_int32()
    sp = SPACES[space] if isinstance(space, str) else space
    _check(lib.rz_reference(dim, degree, sp, ctypes.byref(n), ctypes.byref(Q), None))
    out = np.empty((Q.value, n.value, n.value))
    _check(lib.rz_reference(dim, degree, sp, None, None, _ptr(out, ctypes.c_double)))
    return out


def numbering(coords, cells, degree, space, n_loc):
    """(n_dofs, cell_dofs, patch_ptr, patch_dofs) as the library builds them, host only."""
    m, keep = _mesh(coords, cells)
    sp = SPACES[space] if isinstance(space, str) else space
    nd, npat, nent = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.rz_numbering(ctypes.byref(m), degree, sp, ctypes.byref(nd), None, ctypes.byref(npat),
                            ctypes.byref(nent), None, None))
    cd = np.empty((m.n_cells, n_loc), dtype=np.int32)
    ptr = np.empty(npat.value + 1, dtype=np.int64)
    dofs = np.empty(nent.value, dtype=np.int32)
    _check(lib.rz_numbering(ctypes.byref(m), degree, sp, None, _ptr(cd, ctypes.c_int32), None, None,
                            _ptr(ptr, ctypes.c_int64), _ptr(dofs, ctypes.c_int32)))
    return nd.value, cd, ptr, dofs


def patch_lists(coords, cells, degree, space, decomposition="paper"):
    """(patch_ptr, patch_dofs) of the first patch family rz_setup builds
    under `decomposition`, host only."""
    m, keep = _mesh(coords, cells)
    sp = SPACES[space] if isinstance(space, str) else space
    dec = DECOMPOSITIONS[decomposition] if isinstance(decomposition, str) else decomposition
    npat, nent = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.rz_patch_lists(ctypes.byref(m), degree, sp, dec, ctypes.byref(npat), ctypes.byref(nent), None, None))
    ptr = np.empty(npat.value + 1, dtype=np.int64)
    dofs = np.empty(nent.value, dtype=np.int32)
    _check(lib.rz_patch_lists(ctypes.byref(m), degree, sp, dec, None, None, _ptr(ptr, ctypes.c_int64),
                              _ptr(dofs, ctypes.c_int32)))
    return ptr, dofs


def _info_dict(i, code):
    return dict(status=i.status, iterations=i.iterations, rel_residual=i.rel_residual, cond_estimate=i.cond_estimate,
                solve_ms=i.solve_ms, outer_iterations=i.outer_iterations, setup_ms=i.setup_ms, code=code)


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Problem:
    """A set-up Riesz-map problem on the GPU (rz_setup)."""

    def __init__(self, coords, cells, degree, space, alpha=1.0, beta=1.0, max_iter=1000, precision="fp64",
                 inner_rtol=0.0, pc="hybrid", graphs=True, stream=None, decomposition="paper",
                 dirichlet_facet=None, coarse="exact", mg_meshes=None):
        """dirichlet_facet: None (pure Neumann) or (n_cells, dim + 1) flags, entry
        (c, j) marking the facet of cell c opposite its j-th vertex as Gamma_D.
        coarse: "exact" or "mg" (the V-cycle on W^k over mg_meshes, a list of
        (coords, cells), finest first)."""
        m, keep = _mesh(coords, cells)
        prec = PRECISIONS[precision] if isinstance(precision, str) else precision
        dec = DECOMPOSITIONS[decomposition] if isinstance(decomposition, str) else decomposition
        flags = None
        if dirichlet_facet is not None:
            flags = np.ascontiguousarray(dirichlet_facet, dtype=np.uint8)
            if flags.shape != (m.n_cells, m.dim + 1):
                raise ValueError("dirichlet_facet must have shape (n_cells, dim + 1)")
        levels, keep_mg = None, []
        if mg_meshes is not None:
            levels = (RzMesh * len(mg_meshes))()
            for i, (Xl, Cl) in enumerate(mg_meshes):
                levels[i], kl = _mesh(Xl, Cl)
                keep_mg.append(kl)
        opts = RzOptions(alpha, beta, max_iter, prec, inner_rtol, PCS[pc] if isinstance(pc, str) else pc,
                         0 if graphs else 1, dec, None if flags is None else _ptr(flags, ctypes.c_uint8),
                         COARSE[coarse] if isinstance(coarse, str) else coarse,
                         0 if mg_meshes is None else len(mg_meshes),
                         None if levels is None else ctypes.cast(levels, ctypes.POINTER(RzMesh)))
        h = ctypes.c_void_p()
        self._h = None
        self.space = SPACES[space] if isinstance(space, str) else space
        _check(lib.rz_setup(ctypes.byref(m), degree, self.space, ctypes.byref(opts), _stream(stream), ctypes.byref(h)))
        self._h = h
        nd, ni, nl, Q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.rz_sizes(h, ctypes.byref(nd), ctypes.byref(ni), ctypes.byref(nl), ctypes.byref(Q)))
        self.n_dofs, self.n_interior, self.n_loc, self.Q = nd.value, ni.value, nl.value, Q.value
        self.n_cells = m.n_cells

    def close(self):
        if self._h:
            lib.rz_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _dev(t):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
            raise TypeError("device vectors must be float64 CUDA/HIP tensors")
        return t

    def _cols(self, t):
        self._dev(t)
        if t.dim() == 1:
            if not t.is_contiguous() or t.numel() < self.n_dofs:
                raise ValueError("vector must be contiguous with n_dofs entries")
            return 1, self.n_dofs
        # column-major (n_dofs, n_rhs): stride(0) == 1
        if t.stride(0) != 1 or t.shape[0] < self.n_dofs:
            raise ValueError("matrix must be column-major with n_dofs rows")
        return t.shape[1], t.stride(1)

    def apply_A(self, x, y, stream=None, fp32=False):
        nr, ld = self._cols(x)
        self._cols(y)
        fn = lib.rz_apply_A_fp32 if fp32 else lib.rz_apply_A
        _check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), nr, ld, _stream(stream)))
        return y

    def apply_A_noalloc(self, x, y, stream=None):
        """rz_apply_A_noalloc: y = A x with the library's static work array."""
        nr, ld = self._cols(x)
        self._cols(y)
        _check(lib.rz_apply_A_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), nr, ld,
                                      _stream(stream)))
        return y

    def apply_P(self, r, z, stream=None, fp32=False):
        nr, ld = self._cols(r)
        self._cols(z)
        fn = lib.rz_apply_P_fp32 if fp32 else lib.rz_apply_P
        _check(fn(self._h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()), nr, ld, _stream(stream)))
        return z

    def solve(self, b, x, rtol=1e-10, stream=None, check=True):
        """PCG on A x = b (one column) or A X = B (column-major n_dofs x n_rhs);
        returns the info dict, or a list of dicts for several columns."""
        nr, ld = self._cols(b)
        nr2, ld2 = self._cols(x)
        if nr != nr2 or ld != ld2:
            raise ValueError("b and x need the same shape and leading dimension")
        info = (RzInfo * nr)()
        code = lib.rz_solve(self._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), nr, ld, rtol,
                            info, _stream(stream))
        if check:
            _check(code)
        out = [_info_dict(i, code) for i in info]
        return out[0] if b.dim() == 1 else out

    def set_apply_tiles(self, cells_per_wave, every_apply=False):
        """rz_set_apply_tiles: 16, 32 or 64 cells per wave (0: the default rule)."""
        _check(lib.rz_set_apply_tiles(self._h, int(cells_per_wave), 1 if every_apply else 0))

    def apply_tiles(self):
        c = ctypes.c_int32()
        _check(lib.rz_get_apply_tiles(self._h, ctypes.byref(c)))
        return c.value

    def patch_sets(self):
        """Per patch family: dict(n_patches, max_size, stored_entries, packed_entries, sum_size)."""
        ns = ctypes.c_int32()
        _check(lib.rz_patch_set_info(self._h, 0, ctypes.byref(ns), None, None, None, None, None))
        out = []
        for k in range(ns.value):
            npat, mx, st, pk, sm = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), \
                ctypes.c_int64()
            _check(lib.rz_patch_set_info(self._h, k, None, ctypes.byref(npat), ctypes.byref(mx), ctypes.byref(st),
                                         ctypes.byref(pk), ctypes.byref(sm)))
            out.append(dict(n_patches=npat.value, max_size=mx.value, stored_entries=st.value,
                            packed_entries=pk.value, sum_size=sm.value))
        return out

    def patch_set_apply(self, k, r, z, stream=None):
        """rz_patch_set_apply: z += the patch solves of family k applied to r."""
        nr, ld = self._cols(r)
        self._cols(z)
        _check(lib.rz_patch_set_apply(self._h, k, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()), nr,
                                      ld, _stream(stream)))
        return z

    def dirichlet_dofs(self):
        """The dofs removed by the Dirichlet boundary, ascending."""
        n = ctypes.c_int64()
        _check(lib.rz_dirichlet_dofs(self._h, ctypes.byref(n), None))
        out = np.empty(n.value, dtype=np.int32)
        _check(lib.rz_dirichlet_dofs(self._h, None, _ptr(out, ctypes.c_int32)))
        return out

    def pc_weights(self):
        rho = np.empty(3)
        _check(lib.rz_pc_weights(self._h, _ptr(rho, ctypes.c_double)))
        return rho

    def export_reference(self):
        out = np.empty((self.Q, self.n_loc, self.n_loc))
        _check(lib.rz_export_reference(self._h, _ptr(out, ctypes.c_double)))
        return out

    def export_topology(self):
        npat, nent = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.rz_export_topology(self._h, None, ctypes.byref(npat), ctypes.byref(nent), None, None))
        cd = np.empty((self.n_cells, self.n_loc), dtype=np.int32)
        ptr = np.empty(npat.value + 1, dtype=np.int64)
        dofs = np.empty(nent.value, dtype=np.int32)
        _check(lib.rz_export_topology(self._h, _ptr(cd, ctypes.c_int32), None, None, _ptr(ptr, ctypes.c_int64),
                                      _ptr(dofs, ctypes.c_int32)))
        return cd, ptr, dofs


class Batch:
    """Several set-up problems solved together (rz_batch_create / rz_batch_solve)."""

    def __init__(self, problems):
        self.problems = list(problems)
        hs = (ctypes.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        h = ctypes.c_void_p()
        self._h = None
        _check(lib.rz_batch_create(hs, len(self.problems), ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            lib.rz_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, bs, xs, rtol=1e-10, stream=None, check=True):
        """bs, xs: lists of contiguous float64 device vectors, one per problem."""
        n = len(self.problems)
        if len(bs) != n or len(xs) != n:
            raise ValueError("one b and one x per problem")
        for p, b, x in zip(self.problems, bs, xs):
            for v in (b, x):
                Problem._dev(v)
                if v.dim() != 1 or not v.is_contiguous() or v.numel() != p.n_dofs:
                    raise ValueError("vectors must be contiguous with n_dofs entries")
        bp = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        info = (RzInfo * n)()
        code = lib.rz_batch_solve(self._h, bp, xp, rtol, info, _stream(stream))
        if check:
            _check(code)
        return [_info_dict(i, code) for i in info]



def derivative_reference(k, degree):
    """The reference-cell derivative matrix of the complex (k = 1: grad
    CG_p -> Ned_p; k = 2: curl Ned_p -> RT_p; k = 3: div RT_p -> DG_{p-1}
    in the library's L2-orthonormal basis of P_{p-1}), host only."""
    nt, nf = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.rz_derivative_reference(k, degree, ctypes.byref(nt), ctypes.byref(nf), None))
    D = np.empty((nt.value, nf.value))
    _check(lib.rz_derivative_reference(k, degree, None, None, _ptr(D, ctypes.c_double)))
    return D


class Hodge:
    """Hodge Laplacian on X^{k-1} x X^k (k = 1, 2, 3) with the weighted
    Riesz-map block preconditioner and MINRES (rz_hodge_*).  Vectors:
    contiguous float64 device tensors of n0 + n1 entries, [sigma; u]."""

    def __init__(self, coords, cells, degree, k, gamma=1.0, pc="hybrid", decomposition="paper", max_iter=1000,
                 coarse="exact", mg_meshes=None, stream=None):
        m, keep = _mesh(coords, cells)
        levels, keep_mg = None, []
        if mg_meshes is not None:
            levels = (RzMesh * len(mg_meshes))()
            for i, (Xl, Cl) in enumerate(mg_meshes):
                levels[i], kl = _mesh(Xl, Cl)
                keep_mg.append(kl)
        dec = DECOMPOSITIONS[decomposition] if isinstance(decomposition, str) else decomposition
        opts = RzOptions(1.0, 1.0, max_iter, 0, 0.0, PCS[pc] if isinstance(pc, str) else pc, 0, dec, None,
                         COARSE[coarse] if isinstance(coarse, str) else coarse,
                         0 if mg_meshes is None else len(mg_meshes),
                         None if levels is None else ctypes.cast(levels, ctypes.POINTER(RzMesh)))
        h = ctypes.c_void_p()
        self._h = None
        _check(lib.rz_hodge_setup(ctypes.byref(m), degree, k, gamma, ctypes.byref(opts), _stream(stream),
                                  ctypes.byref(h)))
        self._h = h
        n0, n1 = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.rz_hodge_sizes(h, ctypes.byref(n0), ctypes.byref(n1)))
        self.n0, self.n1 = n0.value, n1.value
        self.n = self.n0 + self.n1

    def close(self):
        if self._h:
            lib.rz_hodge_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t):
        Problem._dev(t)
        if t.dim() != 1 or not t.is_contiguous() or t.numel() != self.n:
            raise ValueError("vectors must be contiguous with n0 + n1 entries")
        return ctypes.c_void_p(t.data_ptr())

    def apply(self, x, y, stream=None):
        _check(lib.rz_hodge_apply(self._h, self._vec(x), self._vec(y), _stream(stream)))
        return y

    def apply_P(self, r, z, stream=None):
        _check(lib.rz_hodge_apply_P(self._h, self._vec(r), self._vec(z), _stream(stream)))
        return z

    def solve(self, b, x, rtol=1e-8, stream=None, check=True):
        info = RzInfo()
        code = lib.rz_hodge_solve(self._h, self._vec(b), self._vec(x), rtol, ctypes.byref(info), _stream(stream))
        if check:
            _check(code)
        return _info_dict(info, code)
