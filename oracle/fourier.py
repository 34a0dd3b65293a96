"""Closed-form solution of the linear periodic problem, mode by mode.

For periodic grids, exp(2 pi i k x) is an eigenvector of Delta_h with
eigenvalue -(4/h^2) sin^2(pi k h) per dimension, so f = nu Delta_h - lambda
acts on Fourier coefficient k as multiplication by sigma_k.  One
collocation step (Sec. 2.1) then maps the coefficient u_hat to stage values
(I - dt sigma_k Q)^{-1} 1 u_hat, and the end value to R(dt sigma_k) u_hat,
with R the Radau IIA stability function.  Independent of the sparse stepper:
no matrices in space, only an FFT and M x M solves per mode.
"""
import numpy as np

from . import radau


def sigma(prob):
    nx = prob["nx"][0]
    hx = prob["length"][0] / nx
    kx = np.arange(nx)
    s = -4.0 / hx ** 2 * np.sin(np.pi * kx / nx) ** 2
    if prob["dim"] == 2:
        ny = prob["nx"][1]
        hy = prob["length"][1] / ny
        ky = np.arange(ny)
        s = s[None, :] + (-4.0 / hy ** 2 * np.sin(np.pi * ky / ny) ** 2)[:, None]
    else:
        s = s[None, :]
    return prob["nu"] * s - prob.get("lambda", 0.0)


def solve_linear_periodic(prob, u0):
    assert prob["bc"] == "periodic"
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    Q = radau.tables(M)["Q"]
    sg = sigma(prob)
    ny, nx = sg.shape
    uh = np.fft.fft2(np.asarray(u0, dtype=np.float64).reshape(ny, nx))
    z = (dt * sg).reshape(-1)
    A = np.eye(M)[None] - z[:, None, None] * Q[None]
    stage = np.linalg.solve(A, np.ones((z.size, M, 1)))[..., 0]  # (K, M)
    U = np.zeros((N, M, ny, nx))
    cur = uh.reshape(-1)
    for n in range(N):
        St = stage * cur[:, None]              # (K, M) complex
        for m in range(M):
            U[n, m] = np.fft.ifft2(St[:, m].reshape(ny, nx)).real
        cur = St[:, M - 1]
    return U


def end_value_periodic(prob, u0):
    """u(T) = U_{N,M} only: the coefficient of mode k is R(dt sigma_k)^N u0_hat(k)
    with R(z) = e_M^T (I - z Q)^{-1} 1 the stability function of the step."""
    assert prob["bc"] == "periodic"
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    Q = radau.tables(M)["Q"]
    sg = sigma(prob)
    ny, nx = sg.shape
    z = (dt * sg).reshape(-1)
    A = np.eye(M)[None] - z[:, None, None] * Q[None]
    R = np.linalg.solve(A, np.ones((z.size, M, 1)))[:, M - 1, 0]
    uh = np.fft.fft2(np.asarray(u0, dtype=np.float64).reshape(ny, nx)).reshape(-1)
    return np.fft.ifft2((R ** N * uh).reshape(ny, nx)).real
