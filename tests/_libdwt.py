"""numpy-FFT form of the DWT on a digital net, used only as an independent pin
of the oracle: by the index identity of Section 2.2 the coefficients are the
m-dimensional DFT of the data over the base-p digit tensor of the point index
(n_0 fastest), which numpy's FFT computes."""
import numpy as np


def lib_dwt(p, m, v):
    N = p ** m
    return np.fft.fftn(np.asarray(v, dtype=np.complex128).reshape([p] * m, order="F")).reshape(N, order="F") / N


def lib_idwt(p, m, ct):
    N = p ** m
    return np.fft.ifftn(np.asarray(ct, dtype=np.complex128).reshape([p] * m, order="F")).reshape(N, order="F") * N
