"""Thin ctypes binding of libmdmrg.so (argument marshalling only).

Every computation happens in the C++/HIP library; this module only converts
numpy arrays / torch device tensors into the plain pointers and sizes of the
C ABI declared in include/mdmrg.h, and turns negative status codes into
exceptions.  Device buffers are torch tensors on the context's device (torch
is used for device memory and streams only).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(HERE, 'libmdmrg.so')

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOCONV, EUNSUP = 0, -1, -2, -3, -4, -5, -6
SPINLESS, HUBBARD = 0, 1
REAL, MOMENTUM = 0, 1
FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
OPT_KEEP_ENVS, OPT_SCRATCH_LIMIT, OPT_GRAPH, OPT_COMPRESS, OPT_GEMM_VARIANT, OPT_MEMORY_BUDGET = 1, 2, 3, 4, 5, 6
OPT_DAVIDSON_KEEP, OPT_DAVIDSON_OLSEN, OPT_MIXED_LADDER, OPT_MIXED_HANDOVER, OPT_MIXED_CORRECT = 7, 8, 9, 10, 11

_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_c_i32_p = ctypes.POINTER(ctypes.c_int32)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)

EXPORTS = {
    'mdmrg_version': (ctypes.c_char_p, []),
    'mdmrg_create': (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p]),
    'mdmrg_destroy': (None, [ctypes.c_void_p]),
    'mdmrg_last_error': (ctypes.c_char_p, [ctypes.c_void_p]),
    'mdmrg_lattice_nso': (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    'mdmrg_build_lattice': (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, _c_dbl_p, _c_dbl_p]),
    'mdmrg_rotate_modes': (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_dbl_p, _c_dbl_p, _c_dbl_p]),
    'mdmrg_set_hamiltonian': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_dbl_p, _c_dbl_p,
                                             ctypes.c_int, ctypes.c_int]),
    'mdmrg_set_hamiltonian_coo': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_dbl_p,
                                                 ctypes.c_int64, _c_i32_p, _c_dbl_p, ctypes.c_int, ctypes.c_int]),
    'mdmrg_n_terms': (ctypes.c_int, [ctypes.c_void_p, _c_i64_p, _c_i64_p]),
    'mdmrg_set_mps': (ctypes.c_int, [ctypes.c_void_p, _c_i32_p, _c_i32_p, _c_i32_p, _c_dbl_p, ctypes.c_int64]),
    'mdmrg_get_bond': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_i32_p, _c_i32_p, _c_i32_p]),
    'mdmrg_set_option': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]),
    'mdmrg_prepare_bond': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    'mdmrg_psi_layout': (ctypes.c_int, [ctypes.c_void_p, _c_i64_p, _c_i32_p, _c_i32_p]),
    'mdmrg_heff_apply': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    'mdmrg_heff_diag': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    'mdmrg_heff_cost': (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, _c_dbl_p, _c_i64_p, _c_i64_p]),
    'mdmrg_heff_histogram': (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p]),
    'mdmrg_davidson': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, _c_dbl_p, _c_dbl_p, ctypes.POINTER(ctypes.c_int)]),
    'mdmrg_davidson_mixed': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_int, ctypes.c_int, _c_dbl_p, _c_dbl_p,
                                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    'mdmrg_decimate': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                      _c_dbl_p, _c_dbl_p, _c_dbl_p]),
    'mdmrg_renormalize': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    'mdmrg_stvec': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    'mdmrg_sweep': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_i32_p, ctypes.c_int, ctypes.c_double,
                                   _c_dbl_p]),
    'mdmrg_gemm_grouped': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                          _c_i64_p, ctypes.c_int64, _c_i64_p, ctypes.c_int64, _c_i64_p,
                                          _c_dbl_p]),
    'mdmrg_gemm_grouped_noalloc': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                                  _c_i64_p, ctypes.c_int64, _c_i64_p, ctypes.c_int64, _c_i64_p,
                                                  _c_dbl_p]),
    'mdmrg_gemm_grouped_split': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_void_p), _c_i64_p, ctypes.c_int64,
                                                _c_i64_p, ctypes.c_int64, _c_i64_p, _c_dbl_p]),
    'mdmrg_get_mps': (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    'mdmrg_get_stats': (ctypes.c_int, [ctypes.c_void_p, _c_dbl_p]),
    'mdmrg_mode_analysis': (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_i32_p, _c_i32_p, _c_i32_p, _c_dbl_p,
                                           ctypes.c_int64, _c_dbl_p, _c_dbl_p, _c_dbl_p, _c_dbl_p, _c_dbl_p,
                                           _c_dbl_p, _c_dbl_p, ctypes.c_int, ctypes.c_int, _c_i32_p, _c_dbl_p,
                                           ctypes.c_int64]),
    'mdmrg_cdw_order': (ctypes.c_int, [ctypes.c_int, _c_dbl_p, _c_dbl_p, _c_dbl_p]),
    'mdmrg_mutual_information': (ctypes.c_int, [ctypes.c_int, _c_dbl_p, _c_dbl_p, _c_i32_p, _c_dbl_p, _c_dbl_p,
                                                _c_dbl_p]),
    'mdmrg_fiedler_order': (ctypes.c_int, [ctypes.c_int, _c_dbl_p, _c_i32_p]),
    'mdmrg_deas_order': (ctypes.c_int, [ctypes.c_int, _c_dbl_p, _c_i32_p]),
    'mdmrg_hf_reference': (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_dbl_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int8)]),
    'mdmrg_natural_orbitals': (ctypes.c_int, [ctypes.c_int, _c_dbl_p, _c_dbl_p, _c_dbl_p]),
    'mdmrg_two_mode_rotation': (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_i32_p, _c_dbl_p, ctypes.c_int64,
                                               ctypes.c_int, _c_dbl_p, _c_dbl_p, _c_dbl_p, _c_dbl_p, _c_dbl_p]),
    'mdmrg_rotation_sweep': (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _c_i32_p, _c_i32_p, _c_i32_p, _c_dbl_p,
                                            ctypes.c_int64, ctypes.c_int, _c_i32_p, _c_dbl_p, ctypes.c_int64,
                                            ctypes.c_int, _c_dbl_p, _c_dbl_p, _c_dbl_p, _c_dbl_p]),
}


class MdmrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f'mdmrg status {code}: {msg}')
        self.code = code


def load(path=None):
    """Load the library and declare the C signatures.  Raises if missing."""
    path = path or DEFAULT_LIB
    if not os.path.exists(path):
        raise RuntimeError(f'libmdmrg not built: {path} is missing (run paper_2311_14106_amd.build)')
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def _dp(a):
    return a.ctypes.data_as(_c_dbl_p)


def _ip(a):
    return a.ctypes.data_as(_c_i32_p)


def device_ptr(t, device, numel, dtype='torch.float64', what='buffer'):
    """Pointer of a device buffer after the checks the C ABI cannot make: a
    contiguous torch tensor on HIP device `device`, of element type `dtype`
    and `numel` elements (None: any length).  Raises ValueError otherwise, so
    that a host array, a tensor on another device, a strided view, a wrong
    element type or a short buffer never reaches a kernel."""
    if isinstance(t, np.ndarray) or not hasattr(t, 'data_ptr'):
        raise ValueError(f'{what}: expected a torch tensor on cuda:{device}, got {type(t).__name__}')
    if not getattr(t, 'is_cuda', False) or t.device.index != device:
        raise ValueError(f'{what}: expected a tensor on cuda:{device}, got one on {t.device}')
    if str(t.dtype) != dtype:
        raise ValueError(f'{what}: expected {dtype}, got {t.dtype}')
    if not t.is_contiguous():
        raise ValueError(f'{what}: tensor must be contiguous')
    if numel is not None and t.numel() != numel:
        raise ValueError(f'{what}: expected {numel} elements, got {t.numel()}')
    return ctypes.c_void_p(t.data_ptr())


def build_lattice(model, basis, Lx, Ly, t, u, L=None):
    L = L or lib()
    nso = L.mdmrg_lattice_nso(model, Lx, Ly)
    T = np.zeros((nso, nso))
    V = np.zeros((nso,) * 4)
    st = L.mdmrg_build_lattice(model, basis, Lx, Ly, t, u, _dp(T), _dp(V))
    if st:
        raise MdmrgError(st, L.mdmrg_last_error(None).decode())
    return T, V


def rotate_modes(R, T, V, spin_half, L=None):
    L = L or lib()
    R = np.ascontiguousarray(R, dtype=np.float64)
    T = np.array(T, dtype=np.float64, order='C')
    V = np.array(V, dtype=np.float64, order='C')
    st = L.mdmrg_rotate_modes(R.shape[0], int(spin_half), _dp(R), _dp(T), _dp(V))
    if st:
        raise MdmrgError(st, L.mdmrg_last_error(None).decode())
    return T, V


def _raw_desc(desc):
    """The (n_blk, 8) int32 block descriptors of mdmrg_psi_layout, from
    either that array or the block list of Context.psi_layout (tuples
    (a, s1, s2, b, offset, m_a, m_b))."""
    if isinstance(desc, np.ndarray):
        return np.ascontiguousarray(desc, dtype=np.int32).reshape(-1, 8)
    out = np.zeros((len(desc), 8), dtype=np.int64)
    for k, (a, s1, s2, b, off, ma, mb) in enumerate(desc):
        out[k] = (a, s1, s2, b, ma, mb, off & 0xFFFFFFFF, off >> 32)
    return out.astype(np.uint32).view(np.int32) if out.size else out.astype(np.int32)


def _host_check(L, st):
    if st:
        raise MdmrgError(st, L.mdmrg_last_error(None).decode())


def mode_analysis(n_sect, sect_qn, sect_dim, data, spin_half, rho=False, centre=None, L=None):
    """One- and two-mode entropies, gamma, occupations and density
    correlations of an MPS in the exchange format (mdmrg_mode_analysis);
    with rho=True also the mode density operators.  centre = (bond, desc,
    psi) replaces the sites bond and bond+1 by the two-site vector psi
    (host array) with the (n_blk, 8) layout desc of psi_layout.  Returns a
    dict of numpy arrays."""
    L = L or lib()
    n_sect = np.ascontiguousarray(n_sect, dtype=np.int32)
    sect_qn = np.ascontiguousarray(sect_qn, dtype=np.int32)
    sect_dim = np.ascontiguousarray(sect_dim, dtype=np.int32)
    data = np.ascontiguousarray(data, dtype=np.float64)
    n = len(n_sect) - 1
    S = int(n_sect.sum())
    if n < 1 or sect_qn.size != 2 * S or sect_dim.size != S:
        raise MdmrgError(EINVAL, 'sector arrays do not match n_sect')
    ns = 2 if spin_half else 1
    d = 1 << ns
    out = {'s_one': np.zeros(n), 's_two': np.zeros((n, n)), 'gamma': np.zeros((n * ns, n * ns)),
           'occ': np.zeros(n * ns), 'nn': np.zeros((n, n))}
    if rho:
        out['rho_one'] = np.zeros((n, d, d))
        out['rho_two'] = np.zeros((n, n, d * d, d * d))
    cb, cdesc, cpsi = -1, None, None
    if centre is not None:
        cb = int(centre[0])
        cdesc = _raw_desc(centre[1])
        cpsi = np.ascontiguousarray(centre[2], dtype=np.float64)
        if cb < 0:
            raise MdmrgError(EINVAL, 'the centre bond must be >= 0')
    st = L.mdmrg_mode_analysis(n, int(bool(spin_half)), _ip(n_sect), _ip(sect_qn), _ip(sect_dim), _dp(data),
                               data.size, _dp(out['s_one']), _dp(out['s_two']),
                               _dp(out['rho_one']) if rho else None, _dp(out['rho_two']) if rho else None,
                               _dp(out['gamma']), _dp(out['occ']), _dp(out['nn']), cb,
                               0 if cdesc is None else cdesc.shape[0], None if cdesc is None else _ip(cdesc),
                               None if cpsi is None else _dp(cpsi), 0 if cpsi is None else cpsi.size)
    _host_check(L, st)
    return out


def cdw_order(nn, signs, L=None):
    """C_CDW from the density correlations of mode_analysis."""
    L = L or lib()
    nn = np.ascontiguousarray(nn, dtype=np.float64)
    signs = np.ascontiguousarray(signs, dtype=np.float64)
    n = signs.size
    if nn.shape != (n, n):
        raise MdmrgError(EINVAL, 'nn must be n x n')
    c = ctypes.c_double()
    _host_check(L, L.mdmrg_cdw_order(n, _dp(nn), _dp(signs), ctypes.byref(c)))
    return c.value


def mutual_information(s_one, s_two, order=None, L=None):
    """(I, I_tot, I_dist) from one- and two-mode entropies."""
    L = L or lib()
    s_one = np.ascontiguousarray(s_one, dtype=np.float64)
    s_two = np.ascontiguousarray(s_two, dtype=np.float64)
    n = s_one.size
    if s_two.shape != (n, n):
        raise MdmrgError(EINVAL, 's_two must be n x n')
    if order is not None:
        order = np.ascontiguousarray(order, dtype=np.int32)
        if order.size != n:
            raise MdmrgError(EINVAL, 'order must list n modes')
    Imat = np.zeros((n, n))
    tot, dist = ctypes.c_double(), ctypes.c_double()
    st = L.mdmrg_mutual_information(n, _dp(s_one), _dp(s_two), _ip(order) if order is not None else None,
                                    _dp(Imat), ctypes.byref(tot), ctypes.byref(dist))
    _host_check(L, st)
    return Imat, tot.value, dist.value


def fiedler_order(Imat, L=None):
    L = L or lib()
    Imat = np.ascontiguousarray(Imat, dtype=np.float64)
    n = Imat.shape[0]
    if Imat.shape != (n, n):
        raise MdmrgError(EINVAL, 'I must be square')
    order = np.zeros(n, dtype=np.int32)
    _host_check(L, L.mdmrg_fiedler_order(n, _dp(Imat), _ip(order)))
    return order


def deas_order(s_one, L=None):
    L = L or lib()
    s_one = np.ascontiguousarray(s_one, dtype=np.float64)
    order = np.zeros(s_one.size, dtype=np.int32)
    _host_check(L, L.mdmrg_deas_order(s_one.size, _dp(s_one), _ip(order)))
    return order


def hf_reference(occ, n_sites, spin_half, target, L=None):
    """0/1 occupation of every spin-orbital of the HF reference."""
    L = L or lib()
    occ = np.ascontiguousarray(occ, dtype=np.float64)
    ns = 2 if spin_half else 1
    if occ.size != n_sites * ns:
        raise MdmrgError(EINVAL, 'occ must hold one value per spin-orbital')
    config = np.zeros(n_sites * ns, dtype=np.int8)
    _host_check(L, L.mdmrg_hf_reference(n_sites, int(bool(spin_half)), _dp(occ), int(target[0]), int(target[1]),
                                        config.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
    return config


def natural_orbitals(gamma, L=None):
    """(occupation numbers descending, natural modes as columns)."""
    L = L or lib()
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    nso = gamma.shape[0]
    if gamma.shape != (nso, nso):
        raise MdmrgError(EINVAL, 'gamma must be square')
    w = np.zeros(nso)
    V = np.zeros((nso, nso))
    _host_check(L, L.mdmrg_natural_orbitals(nso, _dp(gamma), _dp(w), _dp(V)))
    return w, V


def two_mode_rotation(desc, psi, spin_half, thetas=None, rotated=False, L=None):
    """Two-mode micro-iteration at a bond (mdmrg_two_mode_rotation): desc is
    the layout of psi_layout (raw (n_blk, 8) array or block list), psi the
    host vector.
    Returns (theta_best, s_best, s_half at thetas or None, rotated psi or
    None)."""
    L = L or lib()
    desc = _raw_desc(desc)
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    th = None if thetas is None else np.ascontiguousarray(thetas, dtype=np.float64)
    sh = None if th is None else np.zeros(th.size)
    out = np.zeros_like(psi) if rotated else None
    tb, sb = ctypes.c_double(), ctypes.c_double()
    st = L.mdmrg_two_mode_rotation(int(bool(spin_half)), desc.shape[0], _ip(desc), _dp(psi), psi.size,
                                   0 if th is None else th.size, None if th is None else _dp(th),
                                   None if sh is None else _dp(sh), ctypes.byref(tb), ctypes.byref(sb),
                                   None if out is None else _dp(out))
    _host_check(L, st)
    return tb.value, sb.value, sh, out


def rotation_sweep(n_sect, sect_qn, sect_dim, data, spin_half, desc, psi, thetas=None, L=None):
    """Sweep of two-mode micro-iterations from a state with its centre at
    bond 0 (mdmrg_rotation_sweep).  Returns (angles, S_1/2 per bond, R)."""
    L = L or lib()
    n_sect = np.ascontiguousarray(n_sect, dtype=np.int32)
    sect_qn = np.ascontiguousarray(sect_qn, dtype=np.int32)
    sect_dim = np.ascontiguousarray(sect_dim, dtype=np.int32)
    data = np.ascontiguousarray(data, dtype=np.float64)
    n = len(n_sect) - 1
    S = int(n_sect.sum())
    if n < 2 or sect_qn.size != 2 * S or sect_dim.size != S:
        raise MdmrgError(EINVAL, 'sector arrays do not match n_sect')
    desc = _raw_desc(desc)
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    th = None if thetas is None else np.ascontiguousarray(thetas, dtype=np.float64)
    theta = np.zeros(n - 1)
    s_half = np.zeros(n - 1)
    R = np.zeros((n, n))
    st = L.mdmrg_rotation_sweep(n, int(bool(spin_half)), _ip(n_sect), _ip(sect_qn), _ip(sect_dim), _dp(data),
                                data.size, desc.shape[0], _ip(desc), _dp(psi), psi.size,
                                0 if th is None else th.size, None if th is None else _dp(th), _dp(theta),
                                _dp(s_half), _dp(R))
    _host_check(L, st)
    return theta, s_half, R


class Context:
    """One library context on one HIP device."""

    def __init__(self, device=0, path=None, stream=None):
        """stream: a torch.cuda.Stream (or a raw hipStream_t as int) on
        `device` for every device call of the context; None: the library
        creates its own."""
        self.lib = load(path) if path else lib()
        h = ctypes.c_void_p()
        sp = None
        if stream is not None:
            sp = stream if isinstance(stream, int) else stream.cuda_stream
        st = self.lib.mdmrg_create(ctypes.byref(h), device, ctypes.c_void_p(sp) if sp else None)
        if st:
            raise MdmrgError(st, self.lib.mdmrg_last_error(None).decode())
        self.h = h
        self.device = device
        self.stream = stream  # kept alive as long as the context
        self._prev_n_elem = None  # layout length of the bond left by renormalize

    def close(self):
        if self.h:
            self.lib.mdmrg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st, allow=()):
        if st and st not in allow:
            raise MdmrgError(st, self.lib.mdmrg_last_error(self.h).decode())
        return st

    # ---------------------------------------------------------------- model
    def set_hamiltonian(self, n_sites, spin_half, T, V, target):
        T = np.ascontiguousarray(T, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        self._chk(self.lib.mdmrg_set_hamiltonian(self.h, n_sites, int(spin_half), _dp(T), _dp(V),
                                                 int(target[0]), int(target[1])))

    def set_hamiltonian_coo(self, n_sites, spin_half, T, ijkl, val, target):
        T = np.ascontiguousarray(T, dtype=np.float64)
        ijkl = np.ascontiguousarray(ijkl, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        self._chk(self.lib.mdmrg_set_hamiltonian_coo(self.h, n_sites, int(spin_half), _dp(T), len(val),
                                                     _ip(ijkl), _dp(val), int(target[0]), int(target[1])))

    def n_terms(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._chk(self.lib.mdmrg_n_terms(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # ------------------------------------------------------------------ MPS
    def set_mps(self, n_sect, sect_qn, sect_dim, data):
        n_sect = np.ascontiguousarray(n_sect, dtype=np.int32)
        sect_qn = np.ascontiguousarray(sect_qn, dtype=np.int32)
        sect_dim = np.ascontiguousarray(sect_dim, dtype=np.int32)
        data = np.ascontiguousarray(data, dtype=np.float64)
        self._chk(self.lib.mdmrg_set_mps(self.h, _ip(n_sect), _ip(sect_qn), _ip(sect_dim), _dp(data),
                                         len(data)))

    def get_mps(self):
        """Site tensors in the exchange layout of set_mps (flat float64)."""
        n = ctypes.c_int64()
        self._chk(self.lib.mdmrg_get_mps(self.h, None, 0, ctypes.byref(n)))
        data = np.zeros(n.value)
        self._chk(self.lib.mdmrg_get_mps(self.h, _dp(data), len(data), ctypes.byref(n)))
        return data

    def get_bond(self, i):
        n = ctypes.c_int32()
        self._chk(self.lib.mdmrg_get_bond(self.h, i, ctypes.byref(n), None, None))
        qn = np.zeros(2 * n.value, dtype=np.int32)
        dim = np.zeros(n.value, dtype=np.int32)
        self._chk(self.lib.mdmrg_get_bond(self.h, i, ctypes.byref(n), _ip(qn), _ip(dim)))
        return [((int(qn[2 * k]), int(qn[2 * k + 1])), int(dim[k])) for k in range(n.value)]

    # ----------------------------------------------------------------- bond
    def set_option(self, option, value):
        self._chk(self.lib.mdmrg_set_option(self.h, option, int(value)))

    def prepare_bond(self, l):
        self._chk(self.lib.mdmrg_prepare_bond(self.h, l))

    def psi_layout(self):
        ne, nb = ctypes.c_int64(), ctypes.c_int32()
        self._chk(self.lib.mdmrg_psi_layout(self.h, ctypes.byref(ne), ctypes.byref(nb), None))
        desc = np.zeros(8 * nb.value, dtype=np.int32)
        self._chk(self.lib.mdmrg_psi_layout(self.h, ctypes.byref(ne), ctypes.byref(nb), _ip(desc)))
        d = desc.reshape(-1, 8).astype(np.int64)
        off = (d[:, 6] & 0xffffffff) | (d[:, 7] << 32)
        blocks = [(int(a), int(s1), int(s2), int(b), int(o), int(m), int(n))
                  for (a, s1, s2, b, m, n), o in zip(d[:, :6], off)]
        return blocks, ne.value

    def n_elem(self):
        """Length of the current two-site vector (doubles)."""
        ne = ctypes.c_int64()
        self._chk(self.lib.mdmrg_psi_layout(self.h, ctypes.byref(ne), None, None))
        return ne.value

    def _vec(self, t, what, numel=-1):
        return device_ptr(t, self.device, self.n_elem() if numel == -1 else numel, what=what)

    def heff_apply(self, x, y, prec=FP64):
        self._chk(self.lib.mdmrg_heff_apply(self.h, prec, self._vec(x, 'heff_apply x'),
                                            self._vec(y, 'heff_apply y')))

    def heff_diag(self, d):
        self._chk(self.lib.mdmrg_heff_diag(self.h, self._vec(d, 'heff_diag d')))

    def heff_cost(self):
        f, b, t, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._chk(self.lib.mdmrg_heff_cost(self.h, ctypes.byref(f), ctypes.byref(b), ctypes.byref(t),
                                           ctypes.byref(g)))
        return {'flop': f.value, 'bytes': b.value, 'n_terms': t.value, 'n_gemm': g.value}

    HIST_EDGES = (1, 16, 32, 48, 64, 128, 256, 512)
    # tile variants of the grouped kernel (kernel names), in library order
    KERNELS = ('k_gemm', 'k_gemm_w16', 'k_gemm_w4', 'k_gemm_t128')
    N_STATS = 86  # MDMRG_N_STATS

    def heff_histogram(self):
        """{bin lower edge: FLOP} of one H_eff x by min(m, n) of each GEMM."""
        out = np.zeros(8)
        self._chk(self.lib.mdmrg_heff_histogram(self.h, _dp(out)))
        return dict(zip(self.HIST_EDGES, out.tolist()))

    def davidson(self, x, tol=1e-8, max_iter=200, m_max=24):
        e, r, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        st = self._chk(self.lib.mdmrg_davidson(self.h, self._vec(x, 'davidson x'), tol, max_iter, m_max, ctypes.byref(e),
                                               ctypes.byref(r), ctypes.byref(n)), allow=(ENOCONV,))
        return e.value, r.value, n.value, st == OK

    def davidson_mixed(self, x, tol=1e-8, tol_split=1e-5, prec_split=FP32, max_iter=200, m_max=24):
        e, r = ctypes.c_double(), ctypes.c_double()
        n64, ns = ctypes.c_int(), ctypes.c_int()
        st = self._chk(self.lib.mdmrg_davidson_mixed(self.h, self._vec(x, 'davidson_mixed x'), tol, prec_split, tol_split, max_iter, m_max,
                                                     ctypes.byref(e), ctypes.byref(r), ctypes.byref(n64),
                                                     ctypes.byref(ns)), allow=(ENOCONV,))
        return e.value, r.value, n64.value, ns.value, st == OK

    def decimate(self, x, D, direction):
        t, s, h = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.mdmrg_decimate(self.h, self._vec(x, 'decimate x'), D, direction, ctypes.byref(t), ctypes.byref(s),
                                          ctypes.byref(h)))
        return t.value, s.value, h.value

    def renormalize(self, direction, prec=FP64):
        ne = self.n_elem()
        self._chk(self.lib.mdmrg_renormalize(self.h, direction, prec))
        self._prev_n_elem = ne

    def stvec(self, x_old, x_new):
        if self._prev_n_elem is None:
            raise ValueError('stvec: call renormalize first')
        self._chk(self.lib.mdmrg_stvec(self.h, self._vec(x_old, 'stvec x_old', self._prev_n_elem),
                                       self._vec(x_new, 'stvec x_new')))

    def sweep(self, n_sweeps, D_schedule, tol=1e-8, strict=True):
        """Energies after each sweep.  strict: raise when a Davidson solve of
        the sweeps missed tol (ENOCONV); otherwise return them anyway."""
        Ds = np.ascontiguousarray(D_schedule, dtype=np.int32)
        E = np.zeros(n_sweeps)
        self._chk(self.lib.mdmrg_sweep(self.h, n_sweeps, _ip(Ds), len(Ds), tol, _dp(E)),
                  allow=() if strict else (ENOCONV,))
        return E

    def gemm_grouped(self, buffers, out_desc, seg_desc, alpha, prec=FP64):
        """buffers: list of device tensors (float64 for prec FP64, float32 for
        the split forms FP32, BF16X3 and BF16X6); descriptors: int64 arrays of shape
        (n_out, 8) and (n_seg, 8); alpha: float64 (n_seg,)."""
        nb = len(buffers)
        dt = 'torch.float64' if prec == FP64 else 'torch.float32'
        ptrs = (ctypes.c_void_p * nb)(*[device_ptr(b, self.device, None, dt, f'gemm_grouped buffer {i}').value
                                        for i, b in enumerate(buffers)])
        lens = np.array([b.numel() for b in buffers], dtype=np.int64)
        od = np.ascontiguousarray(out_desc, dtype=np.int64).reshape(-1, 8)
        sd = np.ascontiguousarray(seg_desc, dtype=np.int64).reshape(-1, 8)
        al = np.ascontiguousarray(alpha, dtype=np.float64)
        if prec == FP64:
            self._chk(self.lib.mdmrg_gemm_grouped(self.h, nb, ptrs, lens.ctypes.data_as(_c_i64_p), len(od),
                                                  od.ctypes.data_as(_c_i64_p), len(sd),
                                                  sd.ctypes.data_as(_c_i64_p), _dp(al)))
        else:
            self._chk(self.lib.mdmrg_gemm_grouped_split(self.h, prec, nb, ptrs, lens.ctypes.data_as(_c_i64_p),
                                                        len(od), od.ctypes.data_as(_c_i64_p), len(sd),
                                                        sd.ctypes.data_as(_c_i64_p), _dp(al)))

    def gemm_grouped_noalloc(self, buffers, out_desc, seg_desc, alpha):
        """mdmrg_gemm_grouped_noalloc: the FP64 grouped GEMM of gemm_grouped
        with its descriptors staged in the library's static per-GPU array
        (no device allocation); same arguments as gemm_grouped in FP64."""
        nb = len(buffers)
        ptrs = (ctypes.c_void_p * nb)(*[device_ptr(b, self.device, None, 'torch.float64',
                                                   f'gemm_grouped_noalloc buffer {i}').value
                                        for i, b in enumerate(buffers)])
        lens = np.array([b.numel() for b in buffers], dtype=np.int64)
        od = np.ascontiguousarray(out_desc, dtype=np.int64).reshape(-1, 8)
        sd = np.ascontiguousarray(seg_desc, dtype=np.int64).reshape(-1, 8)
        al = np.ascontiguousarray(alpha, dtype=np.float64)
        self._chk(self.lib.mdmrg_gemm_grouped_noalloc(self.h, nb, ptrs, lens.ctypes.data_as(_c_i64_p), len(od),
                                                      od.ctypes.data_as(_c_i64_p), len(sd),
                                                      sd.ctypes.data_as(_c_i64_p), _dp(al)))

    def stats(self):
        out = np.zeros(self.N_STATS)
        self._chk(self.lib.mdmrg_get_stats(self.h, _dp(out)))
        keys = ['diag_h_s', 'ren_s', 'tables_s', 'diag_d_s', 'stvec_s', 'other_s', 'heff_flop', 'n_matvec',
                'heff_gemm_ms', 'heff_gemm_launches', 'heff_gemm_flop',
                'ren_gemm_ms', 'ren_gemm_launches', 'ren_gemm_flop',
                'heff_flop_split', 'n_matvec_split', 'split_gemm_ms', 'split_gemm_launches',
                'split_gemm_flop', 'heff_p1_ms', 'heff_p1_launches', 'heff_p1_flop',
                'grouped_ms', 'grouped_launches', 'grouped_flop',
                'heff_kernel_ms', 'heff_kernel_launches', 'heff_kernel_flop',
                'all_kernel_ms', 'all_kernel_launches']
        for prec in ('f64', 'f32', 'bf3', 'bf6'):
            for var in self.KERNELS:
                keys += [f'proc_{prec}_{var}_ms', f'proc_{prec}_{var}_launches', f'proc_{prec}_{var}_flop']
        keys += ['graph64_ms', 'graph64_launches', 'graph32_ms', 'graph32_launches',
                 'graphbf3_ms', 'graphbf3_launches', 'graphbf6_ms', 'graphbf6_launches']
        assert len(keys) == len(out)
        return dict(zip(keys, out.tolist()))
