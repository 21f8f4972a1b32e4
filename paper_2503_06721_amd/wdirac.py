"""ctypes binding of libwdirac.so.

Argument marshalling only: every computation runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and the current HIP
stream.  Function names are those of the C ABI without the ``wdirac_``
prefix; see include/wdirac.h for the meaning of every argument.

Importing this module raises ImportError if libwdirac.so has not been built
(``__graft_entry__.build()`` or ``python -m paper_2503_06721_amd.build``).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libwdirac.so')
if not os.path.exists(LIB_PATH):
    raise ImportError(f'{LIB_PATH} is not built; run python -m paper_2503_06721_amd.build')
_lib = ctypes.CDLL(LIB_PATH)

# enums of include/wdirac.h
OK, EINVAL, EUNSUPPORTED, EHIP, ENOCONV, EBREAKDOWN = 0, -1, -2, -3, -4, -5
FUND, ADJ, SYM, ASYM = 0, 1, 2, 3
F64, F32 = 0, 1
CG_F64, CG_MIXED = 0, 1
FIELD_HALF_SPINOR, FIELD_LINKS, FIELD_CLOVER = 0, 1, 2
(OP_DHAT, OP_CG, OP_FORCE, OP_NORM, OP_DOT, OP_TUNE, OP_MSHIFT, OP_CLOVER, OP_GAUGE,
 OP_CLOVER_FORCE) = 0, 1, 2, 3, 4, 5, 6, 7, 8, 9
MAX_SHIFTS = 32
(OPT_HOP_VARIANT_F64, OPT_HOP_VARIANT_F32, OPT_XCD_REMAP, OPT_CG_CHECK_EVERY, OPT_MIXED_DELTA, OPT_HOP_NR_F64,
 OPT_HOP_NR_F32, OPT_TILE_TBLOCK, OPT_CG_GRAPH, OPT_TUNE_COMPACT) = 0, 1, 2, 3, 4, 5, 6, 7, 8, 9
HOP_SITE, HOP_COLOUR, HOP_COLOUR_PAIR, HOP_COMPACT, HOP_COMPACT_PAIR, HOP_COLOUR_QUAD, HOP_MULTI = 0, 1, 2, 3, 4, 5, 6
REP_CODES = {'FUND': FUND, 'ADJ': ADJ, 'SYM': SYM, '2AS': ASYM}
STATUS_NAMES = {OK: 'OK', EINVAL: 'EINVAL', EUNSUPPORTED: 'EUNSUPPORTED', EHIP: 'EHIP',
                ENOCONV: 'ENOCONV', EBREAKDOWN: 'EBREAKDOWN'}


class Geom(ctypes.Structure):
    _fields_ = [('dims', ctypes.c_int32 * 4), ('bc', ctypes.c_int32 * 4)]


class Tuning(ctypes.Structure):
    _fields_ = [('variant', ctypes.c_int32), ('nr', ctypes.c_int32), ('xcd_remap', ctypes.c_int32),
                ('tblock', ctypes.c_int32), ('candidates', ctypes.c_int32), ('us', ctypes.c_double),
                ('spread', ctypes.c_double), ('runner_up_us', ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CgStats(ctypes.Structure):
    _fields_ = [('iters', ctypes.c_int32), ('reliable_updates', ctypes.c_int32), ('hops', ctypes.c_int32),
                ('status', ctypes.c_int32), ('true_rel_resid', ctypes.c_double), ('seconds', ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    'wdirac_create': (_I, [ctypes.POINTER(_P), _I, _I, ctypes.POINTER(Geom)]),
    'wdirac_create_batch': (_I, [ctypes.POINTER(_P), _I, _I, ctypes.POINTER(Geom), _I]),
    'wdirac_destroy': (_I, [_P]),
    'wdirac_set_option': (_I, [_P, _I, _D]),
    'wdirac_rep_info': (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    'wdirac_field_bytes': (ctypes.c_size_t, [_P, _I, _I, _I]),
    'wdirac_workspace_bytes': (ctypes.c_size_t, [_P, _I, _I, _I]),
    'wdirac_pack_spinor': (_I, [_P, _P, _P, _I, _I, _I, _P]),
    'wdirac_unpack_spinor': (_I, [_P, _P, _P, _I, _I, _I, _P]),
    'wdirac_rep_links': (_I, [_P, _P, _P, _I, _P]),
    'wdirac_unpack_links': (_I, [_P, _P, _P, _I, _P]),
    'wdirac_dslash_eo': (_I, [_P, _P, _P, _P, _I, _I, _I, _D, _P, _D, _I, _P]),
    'wdirac_apply_Mee': (_I, [_P, _P, _P, _D, _I, _I, _I, _P]),
    'wdirac_apply_Moo': (_I, [_P, _P, _P, _D, _I, _I, _I, _P]),
    'wdirac_apply_dhat': (_I, [_P, _P, _P, _P, _D, _I, _I, _I, _P, _P]),
    'wdirac_eo_source': (_I, [_P, _P, _P, _P, _P, _D, _I, _P]),
    'wdirac_eo_reconstruct': (_I, [_P, _P, _P, _P, _P, _D, _I, _P]),
    'wdirac_norm2': (_I, [_P, ctypes.POINTER(_D), _P, _I, _I, _P, _P]),
    'wdirac_cg_eo': (_I, [_P, _P, _P, _P, _P, _D, _D, _I, _I, _I, _P, ctypes.POINTER(CgStats), _P]),
    'wdirac_dot': (_I, [_P, ctypes.POINTER(_D), _P, _P, _I, _I, _P, _P]),
    'wdirac_force_eo': (_I, [_P, _P, _P, _P, _P, _D, _D, _I, _P, _P]),
    'wdirac_autotune': (_I, [_P, _P, _I, _I, _P, ctypes.POINTER(Tuning), _P]),
    'wdirac_cg_mshift_eo': (_I, [_P, _P, _P, _P, _D, ctypes.POINTER(_D), _I, _D, _I, _P, ctypes.POINTER(CgStats),
                                 _P]),
    'wdirac_axpby': (_I, [_P, _P, _D, _P, _D, _P, _I, _I, _P]),
    'wdirac_gauge_force': (_I, [_P, _P, _P, _D, _D, _I, _P]),
    'wdirac_gauge_action': (_I, [_P, ctypes.POINTER(_D), _P, _D, _P, _P]),
    'wdirac_link_update': (_I, [_P, _P, _P, _D, _P]),
    'wdirac_kinetic': (_I, [_P, ctypes.POINTER(_D), _P, _P, _P]),
    'wdirac_algebra_from_components': (_I, [_P, _P, _P, _P]),
    'wdirac_gamma5': (_I, [_P, _P, _P, _I, _I, _P]),
    'wdirac_apply_W': (_I, [_P, _P, _P, _P, _D, _D, _I, _I, _I, _P, _P]),
    'wdirac_force_bilinear_eo': (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _D, _I, _P]),
    'wdirac_clover_field': (_I, [_P, _P, _P, _D, _D, _I, _I, _P, _P]),
    'wdirac_apply_clover': (_I, [_P, _P, _P, _P, _I, _I, _I, _P]),
    'wdirac_apply_dhat_clover': (_I, [_P, _P, _P, _P, _P, _I, _I, _I, _P, _P]),
    'wdirac_cg_eo_clover': (_I, [_P, _P, _P, _P, _P, _P, _P, _D, _I, _I, _I, _P, ctypes.POINTER(CgStats), _P]),
    'wdirac_force_eo_clover': (_I, [_P, _P, _P, _P, _P, _P, _D, _D, _I, _D, _I, _I, _P, _P]),
    'wdirac_force_clover_logdet': (_I, [_P, _P, _P, _P, _D, _D, _I, _D, _I, _I, _P, _P]),
    'wdirac_clover_logdet': (_I, [_P, ctypes.POINTER(_D), _P, _P, _P]),
    'wdirac_stream_probe': (_I, [_P, ctypes.c_size_t, _I, _I, ctypes.POINTER(_D), _P]),
    'wdirac_apply_dhat_noalloc': (_I, [_P, _P, _P, _P, _D, _I, _I, _I, _P]),
    'wdirac_noalloc_scratch_bytes': (ctypes.c_size_t, []),
    'wdirac_last_error': (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class WdiracError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib.wdirac_last_error().decode()
        super().__init__(f'{where}: {STATUS_NAMES.get(code, code)}: {msg}')


def last_error():
    return _lib.wdirac_last_error().decode()


def _check(code, where, allow=()):
    if code != OK and code not in allow:
        raise WdiracError(code, where)
    return code


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError('libwdirac fields must be GPU tensors')
    if not t.is_contiguous():
        raise ValueError('libwdirac fields must be contiguous')
    return t.data_ptr()


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def stream_probe(elems=1 << 24, nread=7, reps=20, stream=None):
    """GB/s of a pure streaming kernel with nread input streams and one output
    stream of `elems` 16-byte elements (see wdirac_stream_probe)."""
    bufs = torch.empty((nread + 1) * elems * 16, dtype=torch.uint8, device='cuda')
    out = _D()
    _check(_lib.wdirac_stream_probe(_ptr(bufs), elems, nread, reps, ctypes.byref(out), _stream(stream)),
           'stream_probe')
    return out.value


def noalloc_scratch_bytes():
    """Size of the fixed device scratch of apply_dhat_noalloc."""
    return _lib.wdirac_noalloc_scratch_bytes()


class Lattice:
    """A libwdirac context: SU(N) fermions in representation `rep` on `dims`.

    dims = (T, X, Y, Z), bc = per-direction fermion boundary phase (+1/-1).
    A list of shapes, dims = [(T, X, Y, Z), ...], makes a batch of lattices
    processed together (one right-hand side each; canonical batch tensors are
    the per-lattice arrays flattened and concatenated)."""

    def __init__(self, N, rep, dims, bc=(-1, 1, 1, 1)):
        self.N = int(N)
        self.rep_name = rep if isinstance(rep, str) else {v: k for k, v in REP_CODES.items()}[rep]
        self.rep = REP_CODES[self.rep_name] if isinstance(rep, str) else int(rep)
        self.batch = isinstance(dims[0], (tuple, list))
        shapes = [tuple(int(x) for x in dd) for dd in dims] if self.batch else [tuple(int(x) for x in dims)]
        self.shapes = shapes
        self.bc = tuple(int(x) for x in bc)
        geoms = (Geom * len(shapes))(*[Geom((ctypes.c_int32 * 4)(*dd), (ctypes.c_int32 * 4)(*self.bc))
                                         for dd in shapes])
        h = _P()
        _check(_lib.wdirac_create_batch(ctypes.byref(h), self.N, self.rep, geoms, len(shapes)), 'create')
        self._h = h
        self._destroy = _lib.wdirac_destroy   # kept: module globals may be gone when __del__ runs at exit
        d, real = _I(), _I()
        _check(_lib.wdirac_rep_info(h, ctypes.byref(d), ctypes.byref(real)), 'rep_info')
        self.d, self.real = d.value, bool(real.value)
        self.dims = shapes[0] if not self.batch else None
        self.volumes = [dd[0] * dd[1] * dd[2] * dd[3] for dd in shapes]
        self.V = sum(self.volumes)
        self.Vh = self.V // 2
        self.nlat = len(shapes)
        # compact hop forms (fundamental links rebuilt into U_R in registers)
        self.compact = (self.rep_name == 'SYM' and 2 <= self.N <= 4) or (self.rep_name == '2AS' and self.N == 4)

    def nsys(self, nrhs=1):
        """Independent systems of a call: the right-hand sides, or the lattices of a batch."""
        return self.nlat if self.batch else int(nrhs)

    def __del__(self):
        h = getattr(self, '_h', None)
        if h:
            self._destroy(h)
            self._h = None

    # ------------------------------------------------------------ sizes
    def field_bytes(self, kind, nrhs=1, prec=F64):
        return _lib.wdirac_field_bytes(self._h, kind, nrhs, prec)

    def workspace_bytes(self, op, nrhs=1, prec=F64):
        return _lib.wdirac_workspace_bytes(self._h, op, nrhs, prec)

    def set_option(self, option, value):
        _check(_lib.wdirac_set_option(self._h, option, float(value)), 'set_option')

    def new_half(self, nrhs=1, prec=F64, zero=True):
        n = self.field_bytes(FIELD_HALF_SPINOR, nrhs, prec)
        f = torch.zeros if zero else torch.empty
        return f(n, dtype=torch.uint8, device='cuda')

    def new_links(self, prec=F64):
        return torch.empty(self.field_bytes(FIELD_LINKS, 1, prec), dtype=torch.uint8, device='cuda')

    def new_workspace(self, op, nrhs=1, prec=F64):
        return torch.empty(self.workspace_bytes(op, nrhs, prec), dtype=torch.uint8, device='cuda')

    def autotune(self, UR, prec=F64, nrhs=1, workspace=None, stream=None):
        """Time the hop launch shapes for (prec, nrhs) and keep the fastest; returns it."""
        ws = workspace if workspace is not None else self.new_workspace(OP_TUNE, nrhs, prec)
        best = Tuning()
        _check(_lib.wdirac_autotune(self._h, _ptr(UR), prec, nrhs, _ptr(ws), ctypes.byref(best), _stream(stream)),
               'autotune')
        return best.as_dict()

    # ---------------------------------------------------------- layouts
    def pack_spinor(self, packed, canon, parity, nrhs=1, prec=F64, stream=None):
        _check(_lib.wdirac_pack_spinor(self._h, _ptr(packed), _ptr(canon), parity, nrhs, prec, _stream(stream)),
               'pack_spinor')

    def unpack_spinor(self, canon, packed, parity, nrhs=1, prec=F64, stream=None):
        _check(_lib.wdirac_unpack_spinor(self._h, _ptr(canon), _ptr(packed), parity, nrhs, prec, _stream(stream)),
               'unpack_spinor')

    def rep_links(self, UR, U, prec=F64, stream=None):
        _check(_lib.wdirac_rep_links(self._h, _ptr(UR), _ptr(U), prec, _stream(stream)), 'rep_links')

    def unpack_links(self, UR_canon, UR, prec=F64, stream=None):
        _check(_lib.wdirac_unpack_links(self._h, _ptr(UR_canon), _ptr(UR), prec, _stream(stream)), 'unpack_links')

    # --------------------------------------------------------- operators
    def dslash_eo(self, out, inp, UR, out_parity, dagger=0, nrhs=1, alpha=0.0, x_add=None, beta=1.0, prec=F64,
                  stream=None):
        _check(_lib.wdirac_dslash_eo(self._h, _ptr(out), _ptr(inp), _ptr(UR), out_parity, dagger, nrhs,
                                     float(alpha), _ptr(x_add), float(beta), prec, _stream(stream)), 'dslash_eo')

    def apply_Mee(self, out, inp, m0, inverse=0, nrhs=1, prec=F64, stream=None):
        _check(_lib.wdirac_apply_Mee(self._h, _ptr(out), _ptr(inp), float(m0), inverse, nrhs, prec,
                                     _stream(stream)), 'apply_Mee')

    def apply_Moo(self, out, inp, m0, inverse=0, nrhs=1, prec=F64, stream=None):
        _check(_lib.wdirac_apply_Moo(self._h, _ptr(out), _ptr(inp), float(m0), inverse, nrhs, prec,
                                     _stream(stream)), 'apply_Moo')

    def apply_dhat(self, out, inp, UR, m0, dagger=0, nrhs=1, prec=F64, workspace=None, stream=None):
        ws = workspace if workspace is not None else self.new_workspace(OP_DHAT, nrhs, prec)
        _check(_lib.wdirac_apply_dhat(self._h, _ptr(out), _ptr(inp), _ptr(UR), float(m0), dagger, nrhs, prec,
                                      _ptr(ws), _stream(stream)), 'apply_dhat')

    def apply_dhat_noalloc(self, out, inp, UR, m0, dagger=0, nrhs=1, prec=F64, stream=None):
        """apply_dhat without a workspace: the library's fixed scratch array holds the odd field."""
        _check(_lib.wdirac_apply_dhat_noalloc(self._h, _ptr(out), _ptr(inp), _ptr(UR), float(m0), int(dagger),
                                              nrhs, prec, _stream(stream)), 'apply_dhat_noalloc')

    def eo_source(self, b_e, eta_e, eta_o, UR, m0, nrhs=1, stream=None):
        _check(_lib.wdirac_eo_source(self._h, _ptr(b_e), _ptr(eta_e), _ptr(eta_o), _ptr(UR), float(m0), nrhs,
                                     _stream(stream)), 'eo_source')

    def eo_reconstruct(self, psi_o, psi_e, eta_o, UR, m0, nrhs=1, stream=None):
        _check(_lib.wdirac_eo_reconstruct(self._h, _ptr(psi_o), _ptr(psi_e), _ptr(eta_o), _ptr(UR), float(m0),
                                          nrhs, _stream(stream)), 'eo_reconstruct')

    def norm2(self, v, nrhs=1, prec=F64, workspace=None, stream=None):
        ws = workspace if workspace is not None else self.new_workspace(OP_NORM, nrhs, prec)
        out = (_D * self.nsys(nrhs))()
        _check(_lib.wdirac_norm2(self._h, out, _ptr(v), nrhs, prec, _ptr(ws), _stream(stream)), 'norm2')
        return list(out)

    def dot(self, a, b, nrhs=1, prec=F64, workspace=None, stream=None):
        """[<a_k, b_k>] as Python complex numbers."""
        ws = workspace if workspace is not None else self.new_workspace(OP_DOT, nrhs, prec)
        ns = self.nsys(nrhs)
        out = (_D * (2 * ns))()
        _check(_lib.wdirac_dot(self._h, out, _ptr(a), _ptr(b), nrhs, prec, _ptr(ws), _stream(stream)), 'dot')
        return [complex(out[2 * k], out[2 * k + 1]) for k in range(ns)]

    def cg_eo(self, x, b, UR64, m0, tol=1e-10, maxit=10000, nrhs=1, mode=CG_F64, UR32=None, workspace=None,
              stream=None, allow=(ENOCONV, EBREAKDOWN)):
        """Returns (status, [stats dict per rhs])."""
        ws = workspace if workspace is not None else self.new_workspace(OP_CG, nrhs, mode)
        stats = (CgStats * self.nsys(nrhs))()
        rc = _lib.wdirac_cg_eo(self._h, _ptr(x), _ptr(b), _ptr(UR64), _ptr(UR32), float(m0), float(tol),
                               int(maxit), nrhs, mode, _ptr(ws), stats, _stream(stream))
        _check(rc, 'cg_eo', allow)
        return rc, [s.as_dict() for s in stats]

    # ------------------------------------------------------------ HMC pieces
    def gauge_force(self, F, U, beta, scale=1.0, accumulate=0, stream=None):
        _check(_lib.wdirac_gauge_force(self._h, _ptr(F), _ptr(U), float(beta), float(scale), int(accumulate),
                                       _stream(stream)), 'gauge_force')

    def gauge_action(self, U, beta, workspace=None, stream=None):
        ws = workspace if workspace is not None else self.new_workspace(OP_GAUGE)
        out = (_D * self.nlat)()
        _check(_lib.wdirac_gauge_action(self._h, out, _ptr(U), float(beta), _ptr(ws), _stream(stream)),
               'gauge_action')
        return list(out) if self.batch else out[0]

    def link_update(self, U, pi, eps, stream=None):
        _check(_lib.wdirac_link_update(self._h, _ptr(U), _ptr(pi), float(eps), _stream(stream)), 'link_update')

    def kinetic(self, pi, workspace=None, stream=None):
        ws = workspace if workspace is not None else self.new_workspace(OP_GAUGE)
        out = (_D * self.nlat)()
        _check(_lib.wdirac_kinetic(self._h, out, _ptr(pi), _ptr(ws), _stream(stream)), 'kinetic')
        return list(out) if self.batch else out[0]

    def algebra_from_components(self, pi, w, stream=None):
        _check(_lib.wdirac_algebra_from_components(self._h, _ptr(pi), _ptr(w), _stream(stream)),
               'algebra_from_components')

    # ------------------------------------------------ twisted mass, Hasenbusch
    def gamma5(self, out, inp, nrhs=1, prec=F64, stream=None):
        _check(_lib.wdirac_gamma5(self._h, _ptr(out), _ptr(inp), nrhs, prec, _stream(stream)), 'gamma5')

    def apply_W(self, out, inp, UR, m0, mu, sign=1, nrhs=1, prec=F64, workspace=None, stream=None):
        """out = (Q-hat + i sign mu) inp."""
        ws = workspace if workspace is not None else self.new_workspace(OP_DHAT, nrhs, prec)
        _check(_lib.wdirac_apply_W(self._h, _ptr(out), _ptr(inp), _ptr(UR), float(m0), float(mu), int(sign), nrhs,
                                   prec, _ptr(ws), _stream(stream)), 'apply_W')

    def force_bilinear_eo(self, out, X_e, X_o, Y_e, Y_o, UR64, U=None, scale=1.0, accumulate=0, stream=None):
        _check(_lib.wdirac_force_bilinear_eo(self._h, _ptr(out), _ptr(X_e), _ptr(X_o), _ptr(Y_e), _ptr(Y_o),
                                             _ptr(UR64), _ptr(U), float(scale), int(accumulate), _stream(stream)),
               'force_bilinear_eo')

    # ------------------------------------------------------------ clover
    def new_clover(self, prec=F64):
        return torch.empty(self.field_bytes(FIELD_CLOVER, 1, prec), dtype=torch.uint8, device='cuda')

    def clover_field(self, clov, U, m0, csw, exponential=0, prec=F64, workspace=None, stream=None):
        """Clover blocks (D_ee on even sites, D_oo^{-1} on odd sites) from the fundamental links U."""
        ws = workspace if workspace is not None else self.new_workspace(OP_CLOVER, 1, F64)
        _check(_lib.wdirac_clover_field(self._h, _ptr(clov), _ptr(U), float(m0), float(csw), int(exponential),
                                        prec, _ptr(ws), _stream(stream)), 'clover_field')

    def apply_clover(self, out, inp, clov, parity, nrhs=1, prec=F64, stream=None):
        _check(_lib.wdirac_apply_clover(self._h, _ptr(out), _ptr(inp), _ptr(clov), parity, nrhs, prec,
                                        _stream(stream)), 'apply_clover')

    def apply_dhat_clover(self, out, inp, UR, clov, dagger=0, nrhs=1, prec=F64, workspace=None, stream=None):
        ws = workspace if workspace is not None else self.new_workspace(OP_DHAT, nrhs, prec)
        _check(_lib.wdirac_apply_dhat_clover(self._h, _ptr(out), _ptr(inp), _ptr(UR), _ptr(clov), dagger, nrhs,
                                             prec, _ptr(ws), _stream(stream)), 'apply_dhat_clover')

    def cg_eo_clover(self, x, b, UR64, clov64, tol=1e-10, maxit=10000, nrhs=1, mode=CG_F64, UR32=None, clov32=None,
                     workspace=None, stream=None, allow=(ENOCONV, EBREAKDOWN)):
        """Returns (status, [stats dict per system])."""
        ws = workspace if workspace is not None else self.new_workspace(OP_CG, nrhs, mode)
        stats = (CgStats * self.nsys(nrhs))()
        rc = _lib.wdirac_cg_eo_clover(self._h, _ptr(x), _ptr(b), _ptr(UR64), _ptr(UR32), _ptr(clov64), _ptr(clov32),
                                      float(tol), int(maxit), nrhs, mode, _ptr(ws), stats, _stream(stream))
        _check(rc, 'cg_eo_clover', allow)
        return rc, [s.as_dict() for s in stats]

    def force_eo_clover(self, out, x_e, UR64, U, clov64, m0, csw, exponential=0, scale=1.0, gradient=0,
                        accumulate=0, workspace=None, stream=None):
        """Pseudofermion force with the clover D-hat: out = scale * P (or its gradient form 2i P U)."""
        ws = workspace if workspace is not None else self.new_workspace(OP_CLOVER_FORCE, 1, F64)
        _check(_lib.wdirac_force_eo_clover(self._h, _ptr(out), _ptr(x_e), _ptr(UR64), _ptr(U), _ptr(clov64),
                                           float(m0), float(csw), int(exponential), float(scale), int(gradient),
                                           int(accumulate), _ptr(ws), _stream(stream)), 'force_eo_clover')

    def force_clover_logdet(self, out, U, clov64, m0, csw, exponential=0, scale=1.0, gradient=0, accumulate=0,
                            workspace=None, stream=None):
        """Force of S_det = -2 sum_{x odd} log|det D_oo(x)|."""
        ws = workspace if workspace is not None else self.new_workspace(OP_CLOVER_FORCE, 1, F64)
        _check(_lib.wdirac_force_clover_logdet(self._h, _ptr(out), _ptr(U), _ptr(clov64), float(m0), float(csw),
                                               int(exponential), float(scale), int(gradient), int(accumulate),
                                               _ptr(ws), _stream(stream)), 'force_clover_logdet')

    def clover_logdet(self, clov64, workspace=None, stream=None):
        """sum_{x odd} log|det D_oo(x)| (per lattice for a batch)."""
        ws = workspace if workspace is not None else self.new_workspace(OP_CLOVER_FORCE, 1, F64)
        out = (_D * self.nlat)()
        _check(_lib.wdirac_clover_logdet(self._h, out, _ptr(clov64), _ptr(ws), _stream(stream)), 'clover_logdet')
        return list(out) if self.batch else out[0]

    def new_shift_fields(self, nshift):
        """Output buffer of cg_mshift_eo: nshift packed FP64 even fields, one after the other."""
        return torch.zeros(nshift * self.field_bytes(FIELD_HALF_SPINOR, 1, F64), dtype=torch.uint8, device='cuda')

    def shift_field(self, x, k):
        """View of field k of a cg_mshift_eo output buffer."""
        n = self.field_bytes(FIELD_HALF_SPINOR, 1, F64)
        return x[k * n:(k + 1) * n]

    def cg_mshift_eo(self, x, b, UR64, m0, shifts, tol=1e-10, maxit=10000, workspace=None, stream=None,
                     allow=(ENOCONV, EBREAKDOWN)):
        """x_k = (D-hat^+ D-hat + shifts[k])^{-1} b; returns (status, [stats dict per shift])."""
        ns = len(shifts)
        ws = workspace if workspace is not None else self.new_workspace(OP_MSHIFT, ns, F64)
        sh = (_D * ns)(*[float(v) for v in shifts])
        stats = (CgStats * ns)()
        rc = _lib.wdirac_cg_mshift_eo(self._h, _ptr(x), _ptr(b), _ptr(UR64), float(m0), sh, ns, float(tol),
                                      int(maxit), _ptr(ws), stats, _stream(stream))
        _check(rc, 'cg_mshift_eo', allow)
        return rc, [s.as_dict() for s in stats]

    def axpby(self, out, a, x, b=0.0, y=None, nrhs=1, prec=F64, stream=None):
        """out = a x + b y (y None: out = a x)."""
        _check(_lib.wdirac_axpby(self._h, _ptr(out), float(a), _ptr(x), float(b), _ptr(y), nrhs, prec,
                                 _stream(stream)), 'axpby')

    def force_eo(self, out, x_e, UR64, m0, U=None, scale=1.0, accumulate=0, workspace=None, stream=None):
        """out = scale * P (U None) or scale * 2i P U (U given), see include/wdirac.h."""
        ws = workspace if workspace is not None else self.new_workspace(OP_FORCE, 1, F64)
        _check(_lib.wdirac_force_eo(self._h, _ptr(out), _ptr(x_e), _ptr(UR64), _ptr(U), float(m0), float(scale),
                                    accumulate, _ptr(ws), _stream(stream)), 'force_eo')

    # ------------------------------------------------------- conveniences
    def spinor_dtype(self, prec):
        return torch.complex128 if prec == F64 else torch.complex64

    def pack_half(self, canon_full, parity, nrhs=1, prec=F64):
        """New packed half field holding the `parity` sites of a canonical full spinor tensor."""
        out = self.new_half(nrhs, prec)
        self.pack_spinor(out, canon_full.contiguous(), parity, nrhs, prec)
        return out

    def unpack_half(self, packed, parity, nrhs=1, prec=F64, into=None):
        """Canonical full spinor tensor (zeros on the other parity) from a packed half field
        (for a batch: the flat concatenation of the lattices' spinors, shape (V_total, 4, d))."""
        shape = ((nrhs,) + self.dims + (4, self.d)) if not self.batch else (self.V, 4, self.d)
        canon = into if into is not None else torch.zeros(shape, dtype=self.spinor_dtype(prec), device='cuda')
        self.unpack_spinor(canon, packed, parity, nrhs, prec)
        return canon

    def links_canonical(self, UR, prec=F64):
        dt = torch.float64 if self.real else torch.complex128
        shape = (self.dims if not self.batch else (self.V,)) + (4, self.d, self.d)
        out = torch.empty(shape, dtype=dt, device='cuda')
        self.unpack_links(out, UR, prec)
        return out
