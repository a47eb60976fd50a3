"""Material coefficients and the double-grid matrix A_M (Sec. 4.2-4.3).

A material object returns the Fourier coefficients of A (``coeff_A``) and of
A^{-1} (``coeff_B``) at arbitrary integer frequencies k, as complex arrays of
shape (d, d, *k.shape[1:]).  ``double_grid_matrix`` then evaluates eq. MBA_GA:

    A_M(x_M^m) = sum_{n in Z_{2N-1}} omega_M^{mn} Ahat(n),

i.e. the Fourier series of A truncated to Z_{2N-1} and sampled on the M-grid
(M >= 2N-1).  It is NOT a sampling of A itself.
"""

from __future__ import annotations

import numpy as np

from . import fourier, grids


class InclusionComposite:
    """A(x) = A0 + sum_i f_i(x - x_i) A_i (eq. inclcomp), from a ``synth`` descriptor.

    The descriptor gives absolute inclusion conductivities A_in, so A_i = A_in - A0.
    Inclusions must not overlap; then A^{-1}(x) = A0^{-1} + sum_i f_i(x - x_i)
    [(A_in)^{-1} - A0^{-1}], which gives the dual coefficients (Cor. Ga_linsys
    uses B_M built by eq. MBA_GA from the Fourier coefficients of A^{-1}).
    """

    def __init__(self, micro):
        self.d = int(micro["d"])
        self.A0 = np.asarray(micro["A0"], float)
        self.shapes = list(micro["shapes"])
        self.centers = np.asarray(micro["centers"], float)
        self.sizes = np.asarray(micro["sizes"], float)
        self.A_in = np.asarray(micro["A_in"], float)

    def _indicator_hat(self, i, k):
        if self.shapes[i] == "rect":
            f = fourier.rect_hat(k, self.sizes[i])
        elif self.shapes[i] == "tri":
            f = fourier.tri_hat(k, self.sizes[i])
        elif self.shapes[i] == "circ":
            if self.d != 2:
                raise ValueError("circ is a 2D shape")
            f = fourier.circ_hat(k, self.sizes[i][0])
        else:
            raise ValueError(self.shapes[i])
        return f * fourier.shift_phase(k, self.centers[i])

    def _coeff(self, k, base, incs):
        d = self.d
        expand = (...,) + (None,) * (k.ndim - 1)
        zero = np.all(k == 0, axis=0)
        out = np.zeros((d, d) + k.shape[1:], dtype=complex)
        out += base[expand] * zero
        for i, Ai in enumerate(incs):
            out += Ai[expand] * self._indicator_hat(i, k)
        return out

    def coeff_A(self, k):
        return self._coeff(k, self.A0, [a - self.A0 for a in self.A_in])

    def coeff_B(self, k):
        B0 = np.linalg.inv(self.A0)
        return self._coeff(k, B0, [np.linalg.inv(a) - B0 for a in self.A_in])


class GridComposite:
    """Piecewise-constant voxel image (eq. gridcomp with psi = rect_{1/P}).

    Lemma grid_compos: the coefficient at frequency m is |P| psihat(m) Chat(m) with
    Chat(m) = (1/|P|) sum_p omega_P^{-mp} C^p, which is P-periodic in m, so it is
    read at m mod P whether P is larger or smaller than 2N-1 (Remark
    eval_with_FFT).  With psihat(m) = prod_a (1/P_a) sinc(m_a/P_a) the factors of
    |P| cancel.  The image holds either scalar conductivities (shape P: C^p = c^p I)
    or symmetric positive definite matrices (shape P + (d, d): eq. gridcomp with
    C^p in R^{d x d}, one DFT per matrix entry); the dual uses the voxel-wise
    inverse (C^p)^{-1}.
    """

    def __init__(self, micro):
        self.d = int(micro["d"])
        self.P = tuple(int(p) for p in micro["P"])
        self.image = np.asarray(micro["image"], float)
        # an optional second image for the dual side (Lemma bounds_bounds: the
        # primal uses an upper approximation of A, the dual a lower one)
        dual = micro.get("image_dual")
        self.image_dual = self.image if dual is None else np.asarray(dual, float)
        self.tensor = self.image.ndim == self.d + 2
        if self.tensor:
            if self.image.shape != self.P + (self.d, self.d) or self.image_dual.shape != self.image.shape:
                raise ValueError("a tensor image has shape P + (d, d)")
            axes = tuple(range(self.d))
            self._chat_A = grids.dft(self.image, axes=axes)
            self._chat_B = grids.dft(np.linalg.inv(self.image_dual), axes=axes)
        else:
            self._chat_A = grids.dft(self.image)
            self._chat_B = grids.dft(1.0 / self.image_dual)

    def _coeff(self, k, chat):
        idx = tuple(np.mod(k[a], self.P[a]) for a in range(self.d))
        win = np.ones(k.shape[1:])
        for a in range(self.d):
            win = win * fourier.sinc(k[a] / self.P[a])
        if self.tensor:
            # chat[idx] has shape k.shape[1:] + (d, d): entries to the front
            val = np.moveaxis(np.moveaxis(chat[idx], -1, 0), -1, 0)
            return val * win
        eye = np.eye(self.d)[(...,) + (None,) * (k.ndim - 1)]
        return eye * (chat[idx] * win)

    def coeff_A(self, k):
        return self._coeff(k, self._chat_A)

    def coeff_B(self, k):
        return self._coeff(k, self._chat_B)


class FourierSeriesMaterial:
    """A material given directly by callables k -> Ahat(k), k -> Bhat(k) (d,d,...)."""

    def __init__(self, d, fA, fB):
        self.d = d
        self._fA = fA
        self._fB = fB

    def coeff_A(self, k):
        return self._fA(k)

    def coeff_B(self, k):
        return self._fB(k)


def make_material(micro):
    if micro["kind"] == "inclusions":
        return InclusionComposite(micro)
    if micro["kind"] == "voxels":
        return GridComposite(micro)
    raise ValueError(micro["kind"])


def double_grid_matrix(mat, N, M, which="A"):
    """Eq. MBA_GA on the M-grid: entries {(a, b): real array of shape M or None}.

    Fourier coefficients on Z_{2N-1} are placed at index n mod M (zero elsewhere)
    and summed with omega_M^{mn} by an inverse DFT.  Entries whose coefficients
    vanish identically are returned as None.
    """
    d = mat.d
    k = grids.freq_grid(M)
    mask = grids.in_Z(k, [2 * n - 1 for n in N])
    coeff = mat.coeff_A(k) if which == "A" else mat.coeff_B(k)
    out = {}
    for a in range(d):
        for b in range(a, d):
            c = np.where(mask, coeff[a, b], 0.0)
            if not np.any(c):
                out[(a, b)] = out[(b, a)] = None
                continue
            v = grids.idft(c)
            if np.max(np.abs(v.imag)) > 1e-9 * max(1.0, np.max(np.abs(v.real))):
                raise ValueError("A_M is not real: coefficients lack Hermitian symmetry")
            out[(a, b)] = out[(b, a)] = np.ascontiguousarray(v.real)
    return out


def apply_pointwise(AM, x):
    """y_a(x_k) = sum_b A_M,ab(x_k) x_b(x_k) (the material step of Algorithm 2)."""
    d = x.shape[0]
    y = np.zeros_like(x)
    for a in range(d):
        for b in range(d):
            if AM[(a, b)] is not None:
                y[a] += AM[(a, b)] * x[b]
    return y
