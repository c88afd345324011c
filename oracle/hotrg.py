"""FP64 CPU oracle of the HOTRG coarse-graining step and its reverse-mode adjoint.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links this file;
only the test suite, the smoke check and the CPU-baseline leg of the benchmark do.  It shares
no code with the HIP implementation: it is plain NumPy (einsum over BLAS, LAPACK ``eigh``),
written from the paper so that each step can be checked by eye.

What is computed (paper, Supplemental Material B and E):

* Forward.  The HOTRG step (equation labelled ``HOTRGstep`` in SM B and the figure beside it)
  merges an upper tensor T_{x1 x1' y j} and a lower tensor T_{x2 x2' j y'} along their shared
  vertical bond j and compresses the doubled horizontal legs with one isometry w on each side:
      T'_{a b y y'} = sum T_{x1 x1' y j} T_{x2 x2' j y'} w_{x1 x2 a} w_{x1' x2' b}.
  w is taken from a local higher-order SVD of the pair (SM B, sentence after ``HOTRGstep``):
  its columns are the leading eigenvectors of the Gram matrix of the (x1, x2) unfolding of the
  pair, G = M M^T, which factorises as G_{(a c),(b d)} = sum_{jk} A_{a b j k} B_{c d j k} with
  A_{abjk} = sum_{x,y} T_{a x y j} T_{b x y k} and B_{abjk} = sum_{x,y} T_{a x j y} T_{b x k y}.
  The direction alternates every step (main text, Fig. 1(a): renormalise along both axes), the
  tensor is rescaled each step and the logs of the scales are accumulated, and after n steps the
  single tensor's periodic self-trace closes the network (main text, scheme (a): 2^n sites).
* Backward.  The SRG environment recursion (SM B, equation ``SRG``) is the chain rule (SM E,
  equations ``Eeq``, ``Teq``, ``Unify``; SM C, equation ``BP``): the environment of the upper copy
  is the incoming environment contracted with the lower copy and both isometries, and likewise
  for the lower copy; the two copies' contributions add.  Beyond the paper (which keeps w fixed),
  w is differentiated through the eigensolve with the symmetric-eigenvector perturbation formula,
  with 1/(l_j - l_i) broadened to d/(d^2 + eps), d = l_j - l_i.

Readings where the paper is silent (each is also listed in the design notes):
  * internal index order T[l][r][u][d] (the paper's T_{x x' y y'}); inputs arrive as [l][u][r][d];
  * the isometry comes from the left (x1, x2) unfolding; chi' = min(chi, X^2), no threshold;
  * the Gram is symmetrised and divided by its trace before the eigensolve (spectrum in [0, 1]);
  * the per-step scale is the Frobenius norm; in the adjoint it is held constant, which is exact
    because everything downstream of it is log-homogeneous in the rescaled tensor;
  * each step doubles the number of sites, so step k's log-scale carries weight 2^-k and the final
    trace 2^-n (N = 2^n sites);
  * the first step merges a vertical pair (the paper's figure), later steps alternate by the
    permutation (u, d, l, r) of the previous step's output.

The side rule (option side_rule="min"; the default "left" is the reading above).  The local HOSVD
of SM B can be taken on either unfolding of the pair: the left legs (x1, x2) or the right legs
(x1', x2').  For a tensor with the left/right mirror symmetry the two Grams have the same spectrum,
but a chiral tensor (invariant under quarter turns only) gives two different ones.  One bond between
two columns carries a single projector w w^T, so one w serves both sides; the rule takes it from the
unfolding whose discarded eigenvalues weigh less, the truncated weight 1 - sum of the kept
trace-normalised eigenvalues (the choice of the original HOTRG between its two environments).  The
right side wins only when its weight is below the left's by more than SIDE_MARGIN (absolute, on the
trace-normalised spectrum), so that ties decided by rounding always go left.  The right unfolding's
Gram is the left unfolding's Gram of the mirrored step input T[x'][x][y][y'], and its adjoint goes
back through the same transpose.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

DEFAULT_BROADENING = 1e-12
SIDE_MARGIN = 1e-12
SIDE_RULES = ("left", "min")


def _es(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


@dataclass
class StepRecord:
    """What the forward pass keeps of step k for the adjoint and for diagnostics."""
    T: np.ndarray        # normalised input of the step, [l][r][u][d]
    c: float             # Frobenius norm of the unnormalised output
    U: np.ndarray        # all eigenvectors of the normalised Gram, columns sorted descending
    lam: np.ndarray      # eigenvalues of the normalised Gram, descending
    trace_G: float       # trace of the symmetrised Gram
    G_hat: np.ndarray    # symmetrised, trace-normalised Gram
    A: np.ndarray        # half-environment A[a][b][j][k]
    B: np.ndarray        # half-environment B[a][b][j][k]
    chi_kept: int        # chi' = min(chi, X^2)
    P: np.ndarray | None = None
    Q: np.ndarray | None = None
    w_fixed: np.ndarray | None = None   # the step's given isometry (then U, lam, A, B, G_hat are None)
    side: str = "L"      # unfolding the isometry came from: "L" (x1, x2) or "R" (x1', x2')
    trunc_LR: tuple | None = None       # side_rule "min": the truncated weights of both unfoldings


@dataclass
class ForwardResult:
    lnZ_per_site: float
    steps: list
    c0: float
    final_T: np.ndarray
    final_trace: float


def to_internal(T0_lurd: np.ndarray) -> np.ndarray:
    """[l][u][r][d] -> [l][r][u][d]."""
    return np.ascontiguousarray(np.transpose(T0_lurd, (0, 2, 1, 3)))


def half_environments(T: np.ndarray):
    """A[a,b,j,k] = sum_{x,y} T[a,x,y,j] T[b,x,y,k];  B[a,b,j,k] = sum_{x,y} T[a,x,j,y] T[b,x,k,y].

    A pairs two upper copies over their right and up legs (free: left legs a, b and the shared
    vertical legs j, k); B pairs two lower copies over their right and down legs.
    """
    A = _es("axyj,bxyk->abjk", T, T)
    B = _es("axjy,bxky->abjk", T, T)
    return A, B


def gram(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """G[(a,c),(b,d)] = sum_{j,k} A[a,b,j,k] B[c,d,j,k]: Gram of the (x1, x2) unfolding."""
    X = A.shape[0]
    G4 = _es("abjk,cdjk->acbd", A, B)
    return G4.reshape(X * X, X * X)


def isometry(G: np.ndarray, chi: int):
    """Symmetrise, normalise by the trace, full eigendecomposition sorted by descending eigenvalue."""
    Gs = 0.5 * (G + G.T)
    t = float(np.trace(Gs))
    if not (t > 0.0 and math.isfinite(t)):
        raise FloatingPointError("Gram trace is not positive and finite")
    G_hat = Gs / t
    lam, U = np.linalg.eigh(G_hat)
    order = np.argsort(lam)[::-1]
    lam, U = lam[order], U[:, order]
    chi_kept = min(chi, G.shape[0])
    return G_hat, t, lam, U, chi_kept


def mirror_lr(T: np.ndarray) -> np.ndarray:
    """T[x][x'][y][y'] -> T[x'][x][y][y']: the step input seen from its right legs."""
    return np.ascontiguousarray(np.transpose(T, (1, 0, 2, 3)))


def truncated_weight(lam: np.ndarray, chi_kept: int) -> float:
    """1 - sum of the kept eigenvalues of the trace-normalised Gram."""
    return 1.0 - float(np.sum(lam[:chi_kept]))


def project(T: np.ndarray, w: np.ndarray):
    """The HOTRG step with isometry w[x1][x2][a] on both sides, in three pairwise contractions.

    P[i,y,j,b,a] = sum_x1 T[x1,i,y,j] w[x1,b,a]          (upper copy, left isometry)
    Q[i,y,a,m,z] = sum_{b,j} P[i,y,j,b,a] T[b,m,j,z]      (lower copy joined over x2 and j)
    T'[a,c,y,z]  = sum_{i,m} Q[i,y,a,m,z] w[i,m,c]        (right isometry)
    """
    P = _es("xiyj,xba->iyjba", T, w)
    Q = _es("iyjba,bmjz->iyamz", P, T)
    Tn = _es("iyamz,imc->acyz", Q, w)
    return P, Q, Tn


def _spill(arr: np.ndarray, spill_dir, tag: str):
    """Storage only: write arr to spill_dir and return a read-only memory map of it (unchanged values)."""
    if spill_dir is None:
        return arr
    import os
    path = os.path.join(spill_dir, tag + ".npy")
    np.save(path, np.ascontiguousarray(arr))
    return np.load(path, mmap_mode="r")


def hotrg_forward(T0_lurd: np.ndarray, chi: int, n_steps: int, keep_PQ: bool = False,
                  spill_dir=None, progress=None, w_fixed=None, side_rule: str = "left") -> ForwardResult:
    """ln Z / N of the periodic 2^n-site network built from T0 with chi-truncated HOTRG steps.

    spill_dir (optional) keeps each step's record on disk as read-only memory maps instead of in
    RAM; the values are the same, it only lets the largest bond dimensions fit in host memory.
    progress (optional) is called as progress("forward", k) after each step.
    w_fixed (optional) maps step numbers k to given isometries w[x1][x2][a] (chi' = min(chi, X^2)
    columns): those steps project with them instead of the leading eigenvectors of their Gram.
    side_rule: "left" (the (x1, x2) unfolding) or "min" (the unfolding with the smaller truncated
    weight; module notes).
    """
    if side_rule not in SIDE_RULES:
        raise ValueError(f"side_rule must be one of {SIDE_RULES}")
    T0 = np.asarray(T0_lurd, dtype=np.float64)
    if T0.ndim != 4 or len(set(T0.shape)) != 1:
        raise ValueError("T0 must be a D x D x D x D tensor")
    if chi < 1 or n_steps < 1:
        raise ValueError("chi and n_steps must be positive")
    if not np.all(np.isfinite(T0)):
        raise FloatingPointError("T0 has non-finite entries")
    T = to_internal(T0)
    c0 = float(np.linalg.norm(T))
    if not c0 > 0.0:
        raise FloatingPointError("T0 is zero")
    T = T / c0
    L = math.log(c0)
    steps = []
    for k in range(1, n_steps + 1):
        if k > 1:
            T = np.ascontiguousarray(np.transpose(T, (2, 3, 0, 1)))
        X = T.shape[0]
        if w_fixed is not None and k in w_fixed:
            w = np.asarray(w_fixed[k], dtype=np.float64)
            chi_kept = min(chi, X * X)
            if w.shape != (X, X, chi_kept):
                raise ValueError(f"step {k}: isometry must have shape {(X, X, chi_kept)}")
            A = B = G_hat = U = lam = None
            t = math.nan
            side, trunc_LR = "L", None
        else:
            A, B = half_environments(T)
            G_hat, t, lam, U, chi_kept = isometry(gram(A, B), chi)
            side, trunc_LR = "L", None
            if side_rule == "min":
                A_r, B_r = half_environments(mirror_lr(T))
                right = isometry(gram(A_r, B_r), chi)
                trunc_LR = (truncated_weight(lam, chi_kept), truncated_weight(right[2], chi_kept))
                if trunc_LR[1] < trunc_LR[0] - SIDE_MARGIN:
                    side = "R"
                    A, B = A_r, B_r
                    G_hat, t, lam, U, _ = right
                del A_r, B_r, right
            w = U[:, :chi_kept].reshape(X, X, chi_kept)
        P, Q, Tn = project(T, w)
        if not keep_PQ:
            del P, Q
            P = Q = None
        c = float(np.linalg.norm(Tn))
        if not (c > 0.0 and math.isfinite(c)):
            raise FloatingPointError(f"step {k}: output norm is not positive and finite")
        tag = f"step{k:03d}_"
        fixed = w if U is None else None
        steps.append(StepRecord(T=_spill(T, spill_dir, tag + "T"), c=c,
                                U=None if U is None else _spill(U, spill_dir, tag + "U"), lam=lam, trace_G=t,
                                G_hat=None if G_hat is None else _spill(G_hat, spill_dir, tag + "Ghat"),
                                A=None if A is None else _spill(A, spill_dir, tag + "A"),
                                B=None if B is None else _spill(B, spill_dir, tag + "B"),
                                chi_kept=chi_kept, P=P, Q=Q, w_fixed=fixed, side=side, trunc_LR=trunc_LR))
        del A, B, G_hat, U
        T = Tn / c
        L += math.ldexp(math.log(c), -k)
        if progress is not None:
            progress("forward", k)
    tr = float(_es("xxyy->", T))
    if not (tr > 0.0 and math.isfinite(tr)):
        raise FloatingPointError("final trace is not positive and finite")
    L += math.ldexp(math.log(tr), -n_steps)
    return ForwardResult(lnZ_per_site=L, steps=steps, c0=c0, final_T=T, final_trace=tr)


def broadened_inverse_gap(lam: np.ndarray, eps: float) -> np.ndarray:
    """F[i,j] = d / (d^2 + eps) with d = lam[j] - lam[i]; F[i,i] = 0."""
    d = lam[None, :] - lam[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        F = d / (d * d + eps)
    np.fill_diagonal(F, 0.0)
    return F


def eig_adjoint(U: np.ndarray, lam: np.ndarray, chi_kept: int, Ubar_kept: np.ndarray,
                eps: float) -> np.ndarray:
    """Gradient with respect to the symmetric matrix whose eigenvectors are U, given the gradient
    with respect to its leading chi_kept eigenvectors.

    First-order perturbation of eigenvector j of a symmetric matrix: du_j = sum_{i != j} u_i
    (u_i^T dG u_j) / (l_j - l_i).  Its transpose, restricted to symmetric dG, is
    G_bar = U [F o (Om - Om^T) / 2] U^T with Om = U^T U_bar and F the (broadened) inverse gaps.
    U_bar has zero columns for the discarded eigenvectors.
    """
    n = U.shape[0]
    Ubar = np.zeros((n, n))
    Ubar[:, :chi_kept] = Ubar_kept
    Om = U.T @ Ubar
    S = broadened_inverse_gap(lam, eps) * (Om - Om.T) * 0.5
    return U @ S @ U.T


def projection_adjoint(rec: StepRecord, Tn_bar: np.ndarray):
    """Adjoint of the step's projection (the HOTRG step with its isometry held fixed): the gradient
    with respect to the input T through both copies, and the gradient w_bar with respect to the
    isometry w[x1][x2][a] (through both of its occurrences), given the gradient w.r.t. the
    unnormalised output."""
    T = rec.T
    X = T.shape[0]
    chi_kept = rec.chi_kept
    w = rec.w_fixed if rec.w_fixed is not None else rec.U[:, :chi_kept].reshape(X, X, chi_kept)
    if rec.P is not None:
        P, Q = rec.P, rec.Q
    else:
        P, Q, _ = project(T, w)
    # right isometry:  T'[a,c,y,z] = sum Q[i,y,a,m,z] w[i,m,c]
    Q_bar = _es("acyz,imc->iyamz", Tn_bar, w)
    w_bar_R = _es("acyz,iyamz->imc", Tn_bar, Q)
    del Q                                        # (memory only: the chi^5 buffers go after last use)
    # lower copy:  Q[i,y,a,m,z] = sum P[i,y,j,b,a] T[b,m,j,z]
    P_bar = _es("iyamz,bmjz->iyjba", Q_bar, T)
    T_bar_lower = _es("iyjba,iyamz->bmjz", P, Q_bar)
    del Q_bar, P
    # upper copy and left isometry:  P[i,y,j,b,a] = sum T[x,i,y,j] w[x,b,a]
    T_bar_upper = _es("iyjba,xba->xiyj", P_bar, w)
    w_bar_L = _es("xiyj,iyjba->xba", T, P_bar)
    del P_bar
    return T_bar_upper + T_bar_lower, w_bar_L + w_bar_R


def step_adjoint(rec: StepRecord, Tn_bar: np.ndarray, eps: float) -> np.ndarray:
    """Gradient with respect to the step's input T, given the gradient w.r.t. its unnormalised output."""
    T = rec.T
    X = T.shape[0]
    chi_kept = rec.chi_kept
    T_bar_proj, w_bar = projection_adjoint(rec, Tn_bar)
    # the isometry is the leading eigenvectors of G_hat = sym(G) / tr G
    Ubar_kept = w_bar.reshape(X * X, chi_kept)
    Ghat_bar = eig_adjoint(rec.U, rec.lam, chi_kept, Ubar_kept, eps)
    t = rec.trace_G
    Gs_bar = Ghat_bar / t - (np.sum(Ghat_bar * rec.G_hat) / t) * np.eye(X * X)
    G_bar = 0.5 * (Gs_bar + Gs_bar.T)
    G4_bar = G_bar.reshape(X, X, X, X)          # [a][c][b][d]
    A_bar = _es("acbd,cdjk->abjk", G4_bar, rec.B)
    B_bar = _es("acbd,abjk->cdjk", G4_bar, rec.A)
    # the Gram's tensor: T itself, or its mirror when the isometry came from the right unfolding
    Tg = T if rec.side == "L" else mirror_lr(T)
    # A[a,b,j,k] = sum T[a,x,y,j] T[b,x,y,k]  (both factors are the same tensor)
    T_bar_A = _es("abjk,bxyk->axyj", A_bar, Tg) + _es("abjk,axyj->bxyk", A_bar, Tg)
    # B[a,b,j,k] = sum T[a,x,j,y] T[b,x,k,y]
    T_bar_B = _es("abjk,bxky->axjy", B_bar, Tg) + _es("abjk,axjy->bxky", B_bar, Tg)
    T_bar_G = T_bar_A + T_bar_B
    if rec.side == "R":
        T_bar_G = mirror_lr(T_bar_G)
    return T_bar_proj + T_bar_G


def hotrg_backward(fwd: ForwardResult, gbar: float = 1.0, eps: float = DEFAULT_BROADENING,
                   progress=None, w_bar_out=None) -> np.ndarray:
    """d(gbar * lnZ/N)/dT0 in the input layout [l][u][r][d].  progress as in hotrg_forward.
    Steps with a given isometry (w_fixed) contribute only their projection adjoint; their isometry
    gradients d(gbar * lnZ/N)/dw go to the dict w_bar_out[k] when it is given."""
    n = len(fwd.steps)
    D = fwd.final_T.shape
    # final self-trace: L += 2^-n ln sum_{x,y} T[x,x,y,y]
    T_bar = np.zeros(D)
    idx_x = np.arange(D[0])
    idx_y = np.arange(D[2])
    T_bar[idx_x[:, None], idx_x[:, None], idx_y[None, :], idx_y[None, :]] = (
        gbar * math.ldexp(1.0, -n) / fwd.final_trace)
    for k in range(n, 0, -1):
        rec = fwd.steps[k - 1]
        # output was divided by c_k; c_k itself is held constant (exact, see module notes)
        if rec.w_fixed is not None:
            T_in_bar, w_bar = projection_adjoint(rec, T_bar / rec.c)
            if w_bar_out is not None:
                w_bar_out[k] = w_bar
        else:
            T_in_bar = step_adjoint(rec, T_bar / rec.c, eps)
        T_bar = np.transpose(T_in_bar, (2, 3, 0, 1)) if k > 1 else T_in_bar
        if progress is not None:
            progress("backward", k)
    T_bar = T_bar / fwd.c0
    return np.ascontiguousarray(np.transpose(T_bar, (0, 2, 1, 3)))


def lnZ_and_grad(T0_lurd: np.ndarray, chi: int, n_steps: int, eps: float = DEFAULT_BROADENING,
                 side_rule: str = "left"):
    fwd = hotrg_forward(T0_lurd, chi, n_steps, side_rule=side_rule)
    return fwd.lnZ_per_site, hotrg_backward(fwd, 1.0, eps), fwd


def step_invariants(fwd: ForwardResult):
    """Gauge-invariant per-step quantities: scale c_k, kept count, truncated weight, cut gap."""
    out = []
    for rec in fwd.steps:
        lam = rec.lam
        kept = rec.chi_kept
        if lam is None:      # a step with a given isometry has no spectrum
            out.append({"c": rec.c, "chi_kept": kept, "trunc_weight": None, "cut_gap": None, "lam_kept": None})
            continue
        tw = float(np.sum(lam[kept:])) if kept < lam.size else 0.0
        gap = float(lam[kept - 1] - lam[kept]) if kept < lam.size else float("inf")
        out.append({"c": rec.c, "chi_kept": kept, "trunc_weight": tw, "cut_gap": gap,
                    "lam_kept": lam[:kept].copy()})
    return out
