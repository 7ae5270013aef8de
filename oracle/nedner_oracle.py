"""FP64 CPU oracle of the NEDNER reconstruction operator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import or call this
module: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it. It shares no code, tables or constants with the GPU library.

What it computes is the discretised inversion formula with non-equispaced
sensors (eq. (5), Sec. 2) written in physical units, evaluated by direct sums
with exact exponentials: no window, no oversampling and no interpolation.

    modes     j_i in {-N_i/2, ..., N_i/2-1}, k_i = 2 pi j_i / L_i      (Sec. 2)
              l   in {-N3/2, ..., N3/2-1},  kz  = 2 pi l / (N3 d3)
              |K| = sqrt(k1^2 + k2^2 + kz^2),  omega = c sign(l) |K|   (eq. (1))
    NED       G(j,n) = sum_m h_m/(d1 d2) g[m,n] exp(-i k.(y_m - a))    (eq. (5), (9))
    NER       H(j,l) = sum_n G(j,n) exp(-i omega(j,l) t_n)             (eq. (5), (6))
    weight    W(j,l) = 2 c |kz| / |K|   (l != 0),  W(0,0) = 2c,  W(j!=0,0) = 0
    spectrum  F(j,l) = (dt/d3) W(j,l) H(j,l)                           (eq. (1))
    volume    f = Re IDFT_3(F) / (N1 N2 N3), voxel i at (a + i d)       (Sec. 2, last step)

Readings of the paper used here (the paper is garbled or silent on them):
  * eq. (1) with sound speed c: F[f] = 2 c^2 K_z / omega * F[g](K_x, omega),
    which with omega = c sign(K_z)|K| is 2 c |K_z|/|K|; the discrete Riemann
    sums carry dt (time) and 1/(d1 d2 d3) (DFT of f vs. its Fourier transform).
  * data are one-sided in time (t_n = t0 + n dt, n = 0..Nt-1), not mirrored.
  * the 0/0 weight at l = 0: W = 2c on the axis K_x = 0 (its limit), 0 elsewhere.
  * depth step d3 defaults to c Nt dt / N3 (depth range = c T).
  * the output is the real part of the inverse DFT.

The adjoint is taken with respect to the real Euclidean inner products on data
(M x Nt) and volume (N1 x N2 x N3), so that autograd semantics hold.

It also evaluates the forward operator Q of Sec. 2 (initial pressure -> the
trace of the wave equation's solution on the sensor plane) for a volume on the
voxel grid, taken as periodic: each Fourier mode of the volume oscillates as
cos(c |K| t) (the solution with p(., 0) = f and d/dt p(., 0) = 0), so

    trace     (Q v)[m,n] = Re sum_{j,l} V(j,l) cos(c |K(j,l)| t_n) exp(i k.(y_m - a)),
              V = DFT_3(v) / (N1 N2 N3),

and its adjoint. These sums are exact for the periodic grid model; they carry
no sensor weight h_m and no inversion weight.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["Geometry", "geometry", "mode_numbers", "wavenumbers", "omega",
           "weight", "ned", "ner", "spectrum", "volume_from_spectrum",
           "forward", "adjoint", "adjoint_at", "brute_spectrum", "brute_volume",
           "brute_matrix", "spectrum_at", "trace", "trace_adjoint",
           "brute_trace", "corrcoef", "tenenbaum", "tenenbaum_mean", "mip"]

# Memory cap for one block of the exponential matrix (complex128 entries).
_BLOCK_ENTRIES = 1 << 24


@dataclass(frozen=True)
class Geometry:
    """Time grid, sound speed and output voxel grid (Sec. 2 index sets)."""

    nt: int
    t0: float
    dt: float
    c: float
    n1: int
    n2: int
    n3: int
    a1: float
    a2: float
    d1: float
    d2: float
    d3: float

    @property
    def l1(self) -> float:
        return self.n1 * self.d1

    @property
    def l2(self) -> float:
        return self.n2 * self.d2


def geometry(nt, dt, c, n1, n2, n3, t0=0.0, a1=0.0, a2=0.0, d1=0.0, d2=0.0,
             d3=0.0) -> Geometry:
    """Geometry with the defaults: unit aperture and depth range c*Nt*dt."""
    d1 = 1.0 / n1 if d1 == 0.0 else d1
    d2 = 1.0 / n2 if d2 == 0.0 else d2
    d3 = c * nt * dt / n3 if d3 == 0.0 else d3
    return Geometry(int(nt), float(t0), float(dt), float(c), int(n1), int(n2),
                    int(n3), float(a1), float(a2), float(d1), float(d2), float(d3))


def mode_numbers(n: int) -> np.ndarray:
    """Integer mode numbers of a length-n DFT in FFT storage order.

    Index k holds mode k for k < n/2 and mode k - n otherwise, i.e. the set
    {-n/2, ..., n/2-1} of Sec. 2 for even n. A single voxel across an axis
    (the two-dimensional problem, d = 2) carries the mode {0}.
    """
    k = np.arange(n)
    return np.where(k < (n + 1) // 2, k, k - n)


def wavenumbers(geo: Geometry):
    """Physical wavenumbers (k1, k2, kz) of the mode grid, FFT order."""
    k1 = 2.0 * math.pi * mode_numbers(geo.n1) / geo.l1
    k2 = 2.0 * math.pi * mode_numbers(geo.n2) / geo.l2
    kz = 2.0 * math.pi * mode_numbers(geo.n3) / (geo.n3 * geo.d3)
    return k1, k2, kz


def omega(geo: Geometry) -> np.ndarray:
    """omega(j,l) = c sign(l) |K| on the (N1, N2, N3) mode grid (eq. (1))."""
    k1, k2, kz = wavenumbers(geo)
    kk = np.sqrt(k1[:, None, None] ** 2 + k2[None, :, None] ** 2
                 + kz[None, None, :] ** 2)
    return geo.c * np.sign(kz)[None, None, :] * kk


def weight(geo: Geometry) -> np.ndarray:
    """Inversion weight W(j,l) of eq. (1) on the mode grid (see module readings)."""
    k1, k2, kz = wavenumbers(geo)
    kk = np.sqrt(k1[:, None, None] ** 2 + k2[None, :, None] ** 2
                 + kz[None, None, :] ** 2)
    w = np.zeros((geo.n1, geo.n2, geo.n3))
    nz = kz != 0.0
    w[:, :, nz] = 2.0 * geo.c * np.abs(kz[nz])[None, None, :] / kk[:, :, nz]
    w[0, 0, 0] = 2.0 * geo.c
    return w


def _lateral_factors(xy: np.ndarray, geo: Geometry):
    """exp(-i k1 (y1 - a1)) as (N1, M) and exp(-i k2 (y2 - a2)) as (N2, M)."""
    k1, k2, _ = wavenumbers(geo)
    e1 = np.exp(-1j * k1[:, None] * (xy[None, :, 0] - geo.a1))
    e2 = np.exp(-1j * k2[:, None] * (xy[None, :, 1] - geo.a2))
    return e1, e2


def ned(xy, h, g, geo: Geometry) -> np.ndarray:
    """Non-equispaced-data DFT over the sensors (inner sum of eq. (5), eq. (9)).

    G(j1,j2,n) = sum_m h_m/(d1 d2) g[m,n] exp(-i (k1 (y_m1-a1) + k2 (y_m2-a2))).
    The exponential factorises over the two lateral coordinates; the sum over
    m is taken as a matrix product, a block of j1 rows at a time.
    Returns complex128 (N1, N2, Nt), modes in FFT order.
    """
    xy = np.asarray(xy, dtype=np.float64)
    s = np.asarray(h, dtype=np.float64) / (geo.d1 * geo.d2)
    sg = s[:, None] * np.asarray(g, dtype=np.float64)
    e1, e2 = _lateral_factors(xy, geo)
    m = xy.shape[0]
    out = np.empty((geo.n1, geo.n2, geo.nt), dtype=np.complex128)
    rows = max(1, _BLOCK_ENTRIES // max(1, geo.n2 * m))
    for r0 in range(0, geo.n1, rows):
        r1 = min(geo.n1, r0 + rows)
        e = (e1[r0:r1, None, :] * e2[None, :, :]).reshape(-1, m)
        er, ei = np.ascontiguousarray(e.real), np.ascontiguousarray(e.imag)
        blk = (er @ sg) + 1j * (ei @ sg)
        out[r0:r1] = blk.reshape(r1 - r0, geo.n2, geo.nt)
    return out


def ner(G: np.ndarray, geo: Geometry) -> np.ndarray:
    """Non-equispaced-range DFT in time (outer sum of eq. (5), eq. (6)).

    H(j,l) = sum_n G(j,n) exp(-i omega(j,l) t_n), t_n = t0 + n dt, evaluated
    for each (j,l) as the polynomial sum_n G(j,n) z^n in z = exp(-i omega dt)
    by Horner's rule, times exp(-i omega t0). Returns complex128 (N1, N2, N3).
    """
    w = omega(geo)
    out = np.empty((geo.n1, geo.n2, geo.n3), dtype=np.complex128)
    rows = max(1, (1 << 20) // max(1, geo.n2 * geo.n3))
    for r0 in range(0, geo.n1, rows):
        r1 = min(geo.n1, r0 + rows)
        om = w[r0:r1]
        z = np.exp(-1j * om * geo.dt)
        g = G[r0:r1]
        acc = np.broadcast_to(g[:, :, geo.nt - 1, None], om.shape).astype(np.complex128)
        for n in range(geo.nt - 2, -1, -1):
            acc = acc * z + g[:, :, n, None]
        out[r0:r1] = acc * np.exp(-1j * om * geo.t0)
    return out


def spectrum(xy, h, g, geo: Geometry) -> np.ndarray:
    """F(j,l) = (dt/d3) W(j,l) H(j,l): the DFT coefficients of f (eq. (5)).

    complex128 (N1, N2, N3) in FFT order (index k holds mode k mod N).
    """
    G = ned(xy, h, g, geo)
    H = ner(G, geo)
    return (geo.dt / geo.d3) * weight(geo) * H


def spectrum_at(xy, h, g, geo: Geometry, modes) -> np.ndarray:
    """F(j,l) of eq. (5) at the listed modes only, for workloads whose whole
    spectrum is too large to evaluate here.

    `modes` is (S, 3) of storage indices (i1, i2, i3) into the (N1, N2, N3)
    mode grid in FFT order. The sums are those of `ned`, `ner` and `weight`
    restricted to the listed (j, l): the lateral exponential of each listed
    j against every sensor (one product with the data), then the time sum
    with the exact exponential of omega(j,l) t_n. Returns complex128 (S,).
    """
    modes = np.asarray(modes, dtype=np.int64).reshape(-1, 3)
    k1, k2, kz = wavenumbers(geo)
    K1, K2, KZ = k1[modes[:, 0]], k2[modes[:, 1]], kz[modes[:, 2]]
    xy = np.asarray(xy, dtype=np.float64)
    s = np.asarray(h, dtype=np.float64) / (geo.d1 * geo.d2)
    sg = s[:, None] * np.asarray(g, dtype=np.float64)
    ph = K1[:, None] * (xy[None, :, 0] - geo.a1) + K2[:, None] * (xy[None, :, 1] - geo.a2)
    G = np.cos(ph) @ sg - 1j * (np.sin(ph) @ sg)                   # (S, Nt)
    kk = np.sqrt(K1 ** 2 + K2 ** 2 + KZ ** 2)
    om = geo.c * np.sign(KZ) * kk
    tn = geo.t0 + geo.dt * np.arange(geo.nt)
    H = np.sum(G * np.exp(-1j * om[:, None] * tn[None, :]), axis=1)
    W = np.zeros(len(modes))
    nz = KZ != 0.0
    W[nz] = 2.0 * geo.c * np.abs(KZ[nz]) / kk[nz]
    W[(KZ == 0.0) & (kk == 0.0)] = 2.0 * geo.c
    return (geo.dt / geo.d3) * W * H


def volume_from_spectrum(F: np.ndarray) -> np.ndarray:
    """f = Re IDFT_3(F)/(N1 N2 N3), the closing inverse FFT of Sec. 3."""
    return np.fft.ifftn(F).real


def forward(xy, h, g, geo: Geometry) -> np.ndarray:
    """Reconstructed volume (N1, N2, N3), depth fastest, float64."""
    return volume_from_spectrum(spectrum(xy, h, g, geo))


def adjoint(v, xy, h, geo: Geometry) -> np.ndarray:
    """Adjoint of `forward` for the real inner products: volume -> (M, Nt).

    V = DFT_3(v)/(N1 N2 N3); Q = (dt/d3) W V;
    R(j,n) = sum_l Q(j,l) exp(+i omega(j,l) t_n)  (the NER sum transposed,
             stepped over n by multiplying with exp(+i omega dt));
    g'[m,n] = h_m/(d1 d2) Re sum_j exp(+i k.(y_m - a)) R(j,n).
    """
    v = np.asarray(v, dtype=np.float64)
    n_all = geo.n1 * geo.n2 * geo.n3
    Q = (geo.dt / geo.d3) * weight(geo) * (np.fft.fftn(v) / n_all)
    w = omega(geo)
    R = np.empty((geo.n1, geo.n2, geo.nt), dtype=np.complex128)
    p = Q * np.exp(1j * w * geo.t0)
    z = np.exp(1j * w * geo.dt)
    for n in range(geo.nt):
        if n:
            p = p * z
        R[:, :, n] = p.sum(axis=2)
    xy = np.asarray(xy, dtype=np.float64)
    s = np.asarray(h, dtype=np.float64) / (geo.d1 * geo.d2)
    e1, e2 = _lateral_factors(xy, geo)
    m = xy.shape[0]
    out = np.zeros((m, geo.nt))
    rows = max(1, _BLOCK_ENTRIES // max(1, geo.n2 * m))
    for r0 in range(0, geo.n1, rows):
        r1 = min(geo.n1, r0 + rows)
        e = (e1[r0:r1, None, :] * e2[None, :, :]).reshape(-1, m)
        r = R[r0:r1].reshape(-1, geo.nt)
        er, ei = np.ascontiguousarray(e.real), np.ascontiguousarray(e.imag)
        rr, ri = np.ascontiguousarray(r.real), np.ascontiguousarray(r.imag)
        # Re(conj(e)^T r) with e = exp(-i k.y): conj(e) = exp(+i k.y)
        out += er.T @ rr + ei.T @ ri
    return s[:, None] * out


def adjoint_at(v, xy, h, geo: Geometry, time_idx) -> np.ndarray:
    """The adjoint's output at chosen times only: (A* v)[m, n] for every sensor
    of `xy` (a subset of a workload's sensors, with their h) and each index n
    of `time_idx`, for workloads whose whole adjoint is too large to evaluate.

    The sums of `adjoint` restricted to those (m, n): V = DFT_3(v)/(N1 N2 N3),
    Q = (dt/d3) W V, R(j, n) = sum_l Q(j,l) exp(+i omega(j,l) t_n) with the
    exact exponential at each listed t_n, then
    h_m/(d1 d2) Re sum_j exp(+i k.(y_m - a)) R(j, n). Returns (M_sub, len(time_idx)).
    """
    v = np.asarray(v, dtype=np.float64)
    n_all = geo.n1 * geo.n2 * geo.n3
    Q = (geo.dt / geo.d3) * weight(geo) * (np.fft.fftn(v) / n_all)
    w = omega(geo)
    xy = np.asarray(xy, dtype=np.float64)
    s = np.asarray(h, dtype=np.float64) / (geo.d1 * geo.d2)
    e1, e2 = _lateral_factors(xy, geo)          # exp(-i k y), (N1, M) and (N2, M)
    idx = np.asarray(time_idx, dtype=np.int64).ravel()
    out = np.empty((xy.shape[0], idx.size))
    for i, n in enumerate(idx):
        t = geo.t0 + float(n) * geo.dt
        R = (Q * np.exp(1j * w * t)).sum(axis=2)  # (N1, N2)
        # sum_j exp(+i k.y) R(j) = sum_{j1, j2} conj(e1)[j1, m] R[j1, j2] conj(e2)[j2, m]
        out[:, i] = np.real(np.einsum("am,ab,bm->m", np.conj(e1), R, np.conj(e2)))
    return s[:, None] * out


def _abs_k(geo: Geometry) -> np.ndarray:
    """|K(j,l)| on the (N1, N2, N3) mode grid, FFT order."""
    k1, k2, kz = wavenumbers(geo)
    return np.sqrt(k1[:, None, None] ** 2 + k2[None, :, None] ** 2
                   + kz[None, None, :] ** 2)


def trace(v, xy, geo: Geometry) -> np.ndarray:
    """Forward operator Q of Sec. 2 on the periodic voxel grid: volume -> (M, Nt).

    (Q v)[m,n] = Re sum_j exp(+i k_j.(y_m - a)) R(j,n), with
    R(j,n) = sum_l V(j,l) cos(c |K(j,l)| t_n) and V = DFT_3(v)/(N1 N2 N3):
    the wave equation's solution for the initial pressure v (initial velocity
    zero), mode by mode, evaluated on the sensor plane z = 0 at the sensors.
    The cosine is evaluated directly for each t_n.
    """
    v = np.asarray(v, dtype=np.float64)
    n_all = geo.n1 * geo.n2 * geo.n3
    V = np.fft.fftn(v) / n_all
    kk = _abs_k(geo)
    R = np.empty((geo.n1, geo.n2, geo.nt), dtype=np.complex128)
    for n in range(geo.nt):
        t = geo.t0 + n * geo.dt
        R[:, :, n] = (V * np.cos(geo.c * kk * t)).sum(axis=2)
    xy = np.asarray(xy, dtype=np.float64)
    e1, e2 = _lateral_factors(xy, geo)
    m = xy.shape[0]
    out = np.zeros((m, geo.nt))
    rows = max(1, _BLOCK_ENTRIES // max(1, geo.n2 * m))
    for r0 in range(0, geo.n1, rows):
        r1 = min(geo.n1, r0 + rows)
        e = (e1[r0:r1, None, :] * e2[None, :, :]).reshape(-1, m)
        r = R[r0:r1].reshape(-1, geo.nt)
        er, ei = np.ascontiguousarray(e.real), np.ascontiguousarray(e.imag)
        rr, ri = np.ascontiguousarray(r.real), np.ascontiguousarray(r.imag)
        # Re(conj(e)^T r) with e = exp(-i k.y)
        out += er.T @ rr + ei.T @ ri
    return out


def trace_adjoint(d, xy, geo: Geometry) -> np.ndarray:
    """Adjoint of `trace` for the real inner products: (M, Nt) -> volume.

    G(j,n) = sum_m d[m,n] exp(-i k_j.(y_m - a)) (the lateral sum of `ned`
    with unit sensor weights); C(j,l) = sum_n G(j,n) cos(c |K(j,l)| t_n);
    result Re IDFT_3(C) with the 1/(N1 N2 N3) of the inverse DFT.
    """
    G = ned(xy, np.full(len(xy), geo.d1 * geo.d2), d, geo)
    kk = _abs_k(geo)
    C = np.zeros((geo.n1, geo.n2, geo.n3), dtype=np.complex128)
    for n in range(geo.nt):
        t = geo.t0 + n * geo.dt
        C += G[:, :, n, None] * np.cos(geo.c * kk * t)
    return np.fft.ifftn(C).real


# --------------------------------------------------------------------------
# Brute force: every term of eq. (5) with its own exponential, no factorising,
# no Horner, no FFT. For tiny inputs only; it checks the routines above.
# --------------------------------------------------------------------------

def _brute_modes(geo: Geometry):
    j1 = mode_numbers(geo.n1)
    j2 = mode_numbers(geo.n2)
    l = mode_numbers(geo.n3)
    return j1, j2, l


def brute_spectrum(xy, h, g, geo: Geometry) -> np.ndarray:
    """F(j,l) term by term: one exponential of the full phase per (j,l,m,n)."""
    j1s, j2s, ls = _brute_modes(geo)
    times = geo.t0 + geo.dt * np.arange(geo.nt)
    out = np.zeros((geo.n1, geo.n2, geo.n3), dtype=np.complex128)
    for a, j1 in enumerate(j1s):
        for b, j2 in enumerate(j2s):
            for e, l in enumerate(ls):
                k1 = 2.0 * math.pi * j1 / geo.l1
                k2 = 2.0 * math.pi * j2 / geo.l2
                kz = 2.0 * math.pi * l / (geo.n3 * geo.d3)
                kk = math.sqrt(k1 * k1 + k2 * k2 + kz * kz)
                om = geo.c * (0.0 if l == 0 else math.copysign(1.0, l)) * kk
                if l != 0:
                    wgt = 2.0 * geo.c * abs(kz) / kk
                elif j1 == 0 and j2 == 0:
                    wgt = 2.0 * geo.c
                else:
                    wgt = 0.0
                phase = (k1 * (xy[:, 0, None] - geo.a1)
                         + k2 * (xy[:, 1, None] - geo.a2)
                         + om * times[None, :])
                terms = (h[:, None] / (geo.d1 * geo.d2)) * g * np.exp(-1j * phase)
                out[a, b, e] = (geo.dt / geo.d3) * wgt * terms.sum()
    return out


def brute_volume(F: np.ndarray) -> np.ndarray:
    """Re of the explicit inverse DFT sum, one exponential per (i, j, l)."""
    n1, n2, n3 = F.shape
    j1 = mode_numbers(n1)
    j2 = mode_numbers(n2)
    l = mode_numbers(n3)
    out = np.zeros((n1, n2, n3))
    for i1 in range(n1):
        for i2 in range(n2):
            for i3 in range(n3):
                ph = 2.0 * math.pi * (j1[:, None, None] * i1 / n1
                                      + j2[None, :, None] * i2 / n2
                                      + l[None, None, :] * i3 / n3)
                out[i1, i2, i3] = (F * np.exp(1j * ph)).sum().real / (n1 * n2 * n3)
    return out


def brute_matrix(xy, h, geo: Geometry) -> np.ndarray:
    """Dense matrix of the operator (volume entries x data entries), brute force."""
    m = xy.shape[0]
    cols = []
    for idx in range(m * geo.nt):
        e = np.zeros(m * geo.nt)
        e[idx] = 1.0
        F = brute_spectrum(xy, h, e.reshape(m, geo.nt), geo)
        cols.append(brute_volume(F).ravel())
    return np.stack(cols, axis=1)


def brute_trace(v, xy, geo: Geometry) -> np.ndarray:
    """Q v term by term: an explicit DFT of the volume per mode, then one
    cosine and one lateral exponential per (m, n, j, l). Tiny inputs only."""
    v = np.asarray(v, dtype=np.float64)
    j1s, j2s, ls = _brute_modes(geo)
    i1 = np.arange(geo.n1)[:, None, None]
    i2 = np.arange(geo.n2)[None, :, None]
    i3 = np.arange(geo.n3)[None, None, :]
    n_all = geo.n1 * geo.n2 * geo.n3
    m = len(xy)
    out = np.zeros((m, geo.nt))
    for j1 in j1s:
        for j2 in j2s:
            for l in ls:
                coef = (v * np.exp(-2j * math.pi * (j1 * i1 / geo.n1 + j2 * i2 / geo.n2
                                                    + l * i3 / geo.n3))).sum() / n_all
                k1 = 2.0 * math.pi * j1 / geo.l1
                k2 = 2.0 * math.pi * j2 / geo.l2
                kz = 2.0 * math.pi * l / (geo.n3 * geo.d3)
                kk = math.sqrt(k1 * k1 + k2 * k2 + kz * kz)
                for mm in range(m):
                    lat = np.exp(1j * (k1 * (xy[mm, 0] - geo.a1) + k2 * (xy[mm, 1] - geo.a2)))
                    for n in range(geo.nt):
                        t = geo.t0 + n * geo.dt
                        out[mm, n] += (coef * math.cos(geo.c * kk * t) * lat).real
    return out


# --------------------------------------------------------------------------
# Image quality measures of App. B and maximum intensity projections.
# --------------------------------------------------------------------------

def corrcoef(a, b, mask=None) -> float:
    """Correlation coefficient of two images (App. B, eq. (11)):
    Cov(a, b) / sqrt(Var(a) Var(b)) over the elements where mask is true
    (all elements without a mask), with population moments in float64.
    """
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    if mask is not None:
        keep = np.asarray(mask).ravel().astype(bool)
        a, b = a[keep], b[keep]
    da = a - a.mean()
    db = b - b.mean()
    return float(np.sum(da * db) / math.sqrt(np.sum(da * da) * np.sum(db * db)))


def tenenbaum(img, rect=None) -> float:
    """Tenenbaum sharpness of a 2-D image (App. B, eqs. (12)-(13)): the sum
    over pixels of (g * U)^2 + (g^T * U)^2 with g the 3x3 Sobel kernel
    [[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]].

    The sum runs over the pixels (r, c) of rect = (r0, r1, c0, c1) (half-open;
    the whole image without it) whose 3x3 neighbourhood lies inside the image.
    Each pixel's two responses are summed term by term.
    """
    u = np.asarray(img, dtype=np.float64)
    rows, cols = u.shape
    r0, r1, c0, c1 = (0, rows, 0, cols) if rect is None else rect
    r0, c0 = max(r0, 1), max(c0, 1)
    r1, c1 = min(r1, rows - 1), min(c1, cols - 1)
    g = np.array([[-1.0, 0.0, 1.0], [-2.0, 0.0, 2.0], [-1.0, 0.0, 1.0]])
    total = 0.0
    for r in range(r0, r1):
        for c in range(c0, c1):
            patch = u[r - 1:r + 2, c - 1:c + 2]
            gx = float(np.sum(g * patch))
            gy = float(np.sum(g.T * patch))
            total += gx * gx + gy * gy
    return total


def tenenbaum_mean(img, rect=None) -> float:
    """The normalised Tenenbaum measure of App. B: F / N, with F the sum of
    `tenenbaum` and N the number of elements of the image it is taken over
    (the rectangle rect = (r0, r1, c0, c1) as given, the whole image without
    it), so that the measure does not grow with the image size.
    """
    u = np.asarray(img)
    rows, cols = u.shape
    r0, r1, c0, c1 = (0, rows, 0, cols) if rect is None else rect
    count = max(r1 - r0, 0) * max(c1 - c0, 0)
    return tenenbaum(img, rect) / count if count else 0.0


def mip(vol, axis: int) -> np.ndarray:
    """Maximum intensity projection of a volume along `axis`."""
    return np.max(np.asarray(vol), axis=axis)
