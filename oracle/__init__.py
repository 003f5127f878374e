"""FP64 CPU oracle for the conservative spectral collision operator.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product package.  It shares
no code with the HIP library: the arithmetic lives in ``bz_oracle.c`` (plain
C, FP64, OpenMP over the output frequencies as in Sec. 4 of the paper) and in
the small numpy helpers below, each of which cites the passage it follows.

Functions
---------
grid(N, L)                    Sec. 3.1 eq. (meshpoints)
gauss_legendre(n)             quadrature nodes used for eq. (GHat_calc)
radial_rule(lam, L, nq)       Gauss-Jacobi nodes for the radial integral of eq. (GHat_calc)
ghat(xi, zeta, lam, L)        Sec. 2.2 eq. (GHat_calc), cut off at r0 = L, any lam > -3
dft_forward(f, L)             Sec. 2.2 transform, sampled as in Sec. 3.2
dft_inverse(qhat, L)          Sec. 3.2 inverse transform (real part kept)
Oracle(N, L, lam).collide_hat Sec. 3.2 trapezoid-rule weighted convolution
project(Qt, L, rows)          Sec. 3.3 constrained L2 projection (sign read
                              from the stated minimisation problem)
InelasticOracle(N, L, lam, beta)  eq. (GHat_calc) with beta < 1, 4-row projection
Oracle.rk2(f, dt, eps, steps) Sec. 3.1 Heun second-order Runge-Kutta
moments(f, L)                 density, bulk velocity, temperature
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libbz_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_llp = ctypes.POINTER(ctypes.c_longlong)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH) or os.path.getmtime(_LIBPATH) < os.path.getmtime(
            os.path.join(_HERE, "bz_oracle.c")):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.bzo_grid.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.bzo_gauss_legendre.argtypes = [ctypes.c_int, _dp, _dp]
    lib.bzo_ghat.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.bzo_ghat.restype = ctypes.c_double
    lib.bzo_dft_forward.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
    lib.bzo_dft_inverse.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
    lib.bzo_ctx_create.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.bzo_ctx_create.restype = ctypes.c_void_p
    lib.bzo_ctx_create_q.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp]
    lib.bzo_ctx_create_q.restype = ctypes.c_void_p
    lib.bzo_ghat_q.argtypes = [_dp, _dp, ctypes.c_int, _dp, _dp]
    lib.bzo_ghat_q.restype = ctypes.c_double
    lib.bzo_ctx_free.argtypes = [ctypes.c_void_p]
    lib.bzo_ctx_ghat.argtypes = [ctypes.c_void_p, _ip, _ip]
    lib.bzo_ctx_ghat.restype = ctypes.c_double
    lib.bzo_collide_hat.argtypes = [ctypes.c_void_p, _dp, _dp, _llp]
    lib.bzo_project.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
    lib.bzo_collide.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _llp]
    lib.bzo_rk2_homogeneous.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int]
    lib.bzo_num_threads.restype = ctypes.c_int
    lib.bzo_set_mutation.argtypes = [ctypes.c_int]
    lib.bzo_collide_hat_abs.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.bzo_project_rows.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
    lib.bzo_inel_create.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp]
    lib.bzo_inel_create.restype = ctypes.c_void_p
    lib.bzo_inel_free.argtypes = [ctypes.c_void_p]
    lib.bzo_inel_collide_hat.argtypes = [ctypes.c_void_p, _dp, _dp]
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_dp)


def set_mutation(m: int) -> None:
    """Plant a known mistake in the oracle (pin tests only; 0 restores it)."""
    _load().bzo_set_mutation(int(m))


def num_threads() -> int:
    return int(_load().bzo_num_threads())


def grid(N: int, L: float):
    """Mesh of Sec. 3.1: dv = 2L/N, dzeta = pi/L, v_k = dv (k - N/2), zeta_k = dzeta (k - N/2)."""
    v = np.zeros(N)
    z = np.zeros(N)
    dv = ctypes.c_double()
    dz = ctypes.c_double()
    if _load().bzo_grid(N, L, _p(v), _p(z), ctypes.byref(dv), ctypes.byref(dz)):
        raise ValueError("bad grid")
    return v, z, dv.value, dz.value


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    _load().bzo_gauss_legendre(n, _p(x), _p(w))
    return x, w


def radial_rule(lam: float, L: float, nq: int):
    """Gauss-Jacobi rule for int_0^L r^{lam+2} g(r) dr (lam > -3): the weight r^{lam+2} is
    integrated exactly, so the rule converges geometrically in nq for the entire g of
    eq. (GHat_calc) whatever the endpoint behaviour of r^{lam+2}.  Nodes r_i in [0, L] and
    weights that hold r^{lam+2}; the nodes come from scipy (a library routine)."""
    from scipy.special import roots_jacobi
    a = lam + 2.0
    if not a > -1.0:
        raise ValueError("lambda must exceed -3")
    x, w = roots_jacobi(int(nq), 0.0, a)        # weight (1 + x)^a on [-1, 1]
    r = 0.5 * L * (x + 1.0)
    return np.ascontiguousarray(r), np.ascontiguousarray(w * (0.5 * L) ** (a + 1.0))


def _integer_lambda(lam: float) -> bool:
    return lam in (0.0, 1.0)


def ghat(xi, zeta, lam: float, L: float, nq: int = 400, jacobi: bool | None = None) -> float:
    """Ghat(xi, zeta) of eq. (GHat_calc), cut off at r0 = L, by nq-point quadrature:
    Gauss-Legendre with r^{lam+2} in the weights for lam = 0, 1, Gauss-Jacobi otherwise
    (or as `jacobi` says)."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    zeta = np.ascontiguousarray(zeta, dtype=np.float64)
    if jacobi is None:
        jacobi = not _integer_lambda(float(lam))
    if not jacobi:
        return float(_load().bzo_ghat(_p(xi), _p(zeta), lam, L, nq))
    r, w = radial_rule(float(lam), L, nq)
    return float(_load().bzo_ghat_q(_p(xi), _p(zeta), int(nq), _p(r), _p(w)))


def _as_cube(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    N = f.shape[0]
    if f.shape != (N, N, N):
        raise ValueError("expected an (N, N, N) array")
    return f, N


def dft_forward(f, L: float):
    """fhat_k = (2pi)^{-3/2} dv^3 sum_j f_j exp(-i zeta_k . v_j), naive sum per axis."""
    f, N = _as_cube(f)
    out = np.zeros((N, N, N), dtype=np.complex128)
    _load().bzo_dft_forward(N, L, _p(f), out.ctypes.data_as(_dp))
    return out


def dft_inverse(qhat, L: float):
    """Qt_j = Re[(2pi)^{-3/2} dzeta^3 sum_k Qhat_k exp(+i zeta_k . v_j)]; returns (Qt, max |Im|)."""
    qhat = np.ascontiguousarray(qhat, dtype=np.complex128)
    N = qhat.shape[0]
    out = np.zeros((N, N, N))
    mi = ctypes.c_double()
    _load().bzo_dft_inverse(N, L, qhat.ctypes.data_as(_dp), _p(out), ctypes.byref(mi))
    return out, mi.value


def project(qt, L: float, rows: int = 5):
    """Q = Qt - C^T (C C^T)^{-1} C Qt (Sec. 3.3, Gaussian elimination) with the first `rows`
    constraints: 5 (mass, momentum, energy) for elastic collisions, 4 without the energy
    row for inelastic ones."""
    qt, N = _as_cube(qt)
    out = np.zeros_like(qt)
    lam = np.zeros(5)
    if _load().bzo_project_rows(N, L, int(rows), _p(qt), _p(out), _p(lam)):
        raise RuntimeError("singular constraint Gram matrix")
    return out


class Oracle:
    """Per-mesh oracle context: the Ghat quadrature is memoised on creation."""

    def __init__(self, N: int, L: float, lam: float, nq: int = 400, jacobi: bool | None = None):
        self.N, self.L, self.lam = N, float(L), float(lam)
        if jacobi is None:
            jacobi = not _integer_lambda(self.lam)
        if jacobi:
            r, w = radial_rule(self.lam, self.L, nq)
            self._h = _load().bzo_ctx_create_q(N, self.L, self.lam, int(nq), _p(r), _p(w))
        else:
            self._h = _load().bzo_ctx_create(N, self.L, self.lam, nq)
        if not self._h:
            raise ValueError("bad oracle parameters")

    def __del__(self):
        if getattr(self, "_h", None):
            _load().bzo_ctx_free(self._h)
            self._h = None

    def ghat_idx(self, k, m) -> float:
        """Ghat(xi_m, zeta_k) for mesh index triples k, m."""
        k = (ctypes.c_int * 3)(*[int(x) for x in k])
        m = (ctypes.c_int * 3)(*[int(x) for x in m])
        return float(_load().bzo_ctx_ghat(self._h, k, m))

    def collide_hat(self, fhat):
        """Qhat on the Fourier mesh; returns (Qhat, number of pairs summed)."""
        fhat = np.ascontiguousarray(fhat, dtype=np.complex128)
        out = np.zeros_like(fhat)
        pairs = ctypes.c_longlong()
        _load().bzo_collide_hat(self._h, fhat.ctypes.data_as(_dp), out.ctypes.data_as(_dp),
                                ctypes.byref(pairs))
        return out, int(pairs.value)

    def kappa(self, f) -> float:
        """Cancellation factor ||sum_m |G fhat_m fhat_j| || / ||Qhat|| of the convolution of f."""
        fh = dft_forward(f, self.L)
        qh, _ = self.collide_hat(fh)
        a = np.zeros(fh.shape)
        _load().bzo_collide_hat_abs(self._h, fh.ctypes.data_as(_dp), _p(a))
        return float(np.linalg.norm(a) / max(np.linalg.norm(qh), 1e-300))

    def collide(self, f):
        """f -> (Qt unprojected, Q projected, max |Im| of the inverse transform, pairs)."""
        f, N = _as_cube(f)
        if N != self.N:
            raise ValueError("mesh size mismatch")
        qt = np.zeros_like(f)
        q = np.zeros_like(f)
        mi = ctypes.c_double()
        pairs = ctypes.c_longlong()
        if _load().bzo_collide(self._h, _p(f), _p(qt), _p(q), ctypes.byref(mi), ctypes.byref(pairs)):
            raise RuntimeError("oracle collide failed")
        return qt, q, mi.value, int(pairs.value)

    def rk2(self, f, dt: float, eps: float, steps: int):
        """Heun RK2 on df/dt = Q(f,f)/eps for one cell or a stack of cells (in a copy)."""
        f = np.array(f, dtype=np.float64, copy=True, order="C")
        cells = 1 if f.ndim == 3 else f.shape[0]
        if _load().bzo_rk2_homogeneous(self._h, _p(f), cells, dt, eps, steps):
            raise RuntimeError("oracle rk2 failed")
        return f


class InelasticOracle:
    """Collision operator with the restitution factor beta of eq. (G_eqn) kept in the weights
    of eq. (GHat_calc) (beta = 1 elastic, beta < 1 inelastic; Sec. 3.3: such collisions do
    not preserve energy, so the projection keeps mass and momentum only)."""

    def __init__(self, N: int, L: float, lam: float, beta: float, nq: int = 400):
        self.N, self.L, self.lam, self.beta = N, float(L), float(lam), float(beta)
        r, w = radial_rule(self.lam, self.L, nq)
        self._h = _load().bzo_inel_create(N, self.L, self.beta, int(nq), _p(r), _p(w))
        if not self._h:
            raise ValueError("bad oracle parameters")

    def __del__(self):
        if getattr(self, "_h", None):
            _load().bzo_inel_free(self._h)
            self._h = None

    def collide_hat(self, fhat):
        fhat = np.ascontiguousarray(fhat, dtype=np.complex128)
        out = np.zeros_like(fhat)
        _load().bzo_inel_collide_hat(self._h, fhat.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
        return out

    def collide(self, f):
        """f -> (Qt unprojected, Q projected onto mass and momentum (energy too if beta = 1))."""
        f, N = _as_cube(f)
        qt, _ = dft_inverse(self.collide_hat(dft_forward(f, self.L)), self.L)
        return qt, project(qt, self.L, 5 if self.beta == 1.0 else 4)


def moments(f, L: float):
    """Density, bulk velocity and temperature of a cell (uniform weights dv^3).

    rho = sum f dv^3, u = sum v f dv^3 / rho, T_d = sum (v_d - u_d)^2 f dv^3 / rho,
    T = (T_1 + T_2 + T_3) / 3 (non-dimensional, R = 1).
    """
    f, N = _as_cube(f)
    v, _, dv, _ = grid(N, L)
    w = dv ** 3
    V = np.meshgrid(v, v, v, indexing="ij")
    rho = f.sum() * w
    u = np.array([(V[d] * f).sum() * w / rho for d in range(3)])
    Td = np.array([((V[d] - u[d]) ** 2 * f).sum() * w / rho for d in range(3)])
    return rho, u, Td.mean(), Td
