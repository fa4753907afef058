"""CPU oracle for the randomized UTV factorization (randUTV) -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It shares no code with the HIP path.

What it computes (the paper's Section 3.2): A = U T V^T for a square n x n A
with U, V orthogonal and T upper triangular, built b columns at a time.  With
T := A, U := I, V := I, step i (k0 = i b, the trailing block T22 = T[k0:, k0:]):

1. (V_alpha) Y = (T22^T T22)^q T22^T G_i with the Gaussian draw G_i
   ((n - k0) x b, an input: G[k0:, k0:k0+b] of the caller's n x n G);
   Householder QR of Y (oracle/qr.py, LAPACK conventions); Qy = H_1 ... H_b
   (the full (n-k0) x (n-k0) orthogonal factor).  T[:, k0:] := T[:, k0:] Qy,
   V[:, k0:] := V[:, k0:] Qy.
2. (U_alpha) Householder QR of T22[:, :b]; Qu its full orthogonal factor.
   T[k0:, k0:] := Qu^T T[k0:, k0:] (the block column's entries below the
   diagonal become zero), U[:, k0:] := U[:, k0:] Qu.
3. (U_beta, V_beta) SVD of the b x b block T[k0:k0+b, k0:k0+b] = Us D Vs^T
   (singular values in decreasing order): the block becomes diag(D),
   T[k0:k0+b, k0+b:] := Us^T T[k0:k0+b, k0+b:], T[:k0, k0:k0+b] :=
   T[:k0, k0:k0+b] Vs, U[:, k0:k0+b] := U[:, k0:k0+b] Us, V[:, k0:k0+b] :=
   V[:, k0:k0+b] Vs.
The last step, when at most b columns remain, is only step 3 on the whole
remaining block (its SVD makes it diagonal).

The SVD of the small block is numpy's (LAPACK); its singular vectors are
fixed up to sign, so two correct runs can differ by the sign of a row of T
and of the matching column of U (and of a column of T and of V): checks
compare what is unique (|T|, |U|, |V| entrywise, the diagonal of T).
"""
from __future__ import annotations

import numpy as np

from . import qr


def randutv(A: np.ndarray, b: int, q: int, G: np.ndarray):
    """(U, T, V) with A = U T V^T; G is n x n (step i uses G[k0:, k0:k0+b])."""
    T = np.array(A, dtype=np.float64, copy=True)
    n = T.shape[0]
    assert T.shape == (n, n) and G.shape[0] >= n and G.shape[1] >= n
    U = np.eye(n)
    V = np.eye(n)
    for k0 in range(0, n, b):
        nr = n - k0
        if nr > b:
            T22 = T[k0:, k0:]
            Y = T22.T @ G[k0:, k0:k0 + b]
            for _ in range(q):
                Y = T22.T @ (T22 @ Y)
            F, tau = qr.geqr2(Y)
            Qy = qr.form_q(F, tau, nr)
            T[:, k0:] = T[:, k0:] @ Qy
            V[:, k0:] = V[:, k0:] @ Qy
            F, tau = qr.geqr2(T[k0:, k0:k0 + b])
            Qu = qr.form_q(F, tau, nr)
            T[k0:, k0:] = Qu.T @ T[k0:, k0:]
            T[k0 + b:, k0:k0 + b] = 0.0
            U[:, k0:] = U[:, k0:] @ Qu
            w = b
        else:
            w = nr
        Us, D, Vst = np.linalg.svd(T[k0:k0 + w, k0:k0 + w])
        Vs = Vst.T
        T[k0:k0 + w, k0:k0 + w] = np.diag(D)
        if k0 + w < n:
            T[k0:k0 + w, k0 + w:] = Us.T @ T[k0:k0 + w, k0 + w:]
        if k0:
            T[:k0, k0:k0 + w] = T[:k0, k0:k0 + w] @ Vs
        U[:, k0:k0 + w] = U[:, k0:k0 + w] @ Us
        V[:, k0:k0 + w] = V[:, k0:k0 + w] @ Vs
    return U, T, V
