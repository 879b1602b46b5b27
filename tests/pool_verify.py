"""Verification of GPU GEMM outputs at full workload sizes against the FP64 oracle (test
infrastructure).

Every output gets three checks, each against expected values that only the oracle computes:
  * a Freivalds row check with two seeded sign vectors X: C X (reduced on the device from the
    GPU's own output) against A (B X), bounded by tol |A| (|B| |X|) (oracle.check);
  * 4,096 sampled entries (64 seeded rows x 64 seeded columns) against C_ref with the
    problem statement's error measure |C - C_ref| / (|A||B|);
  * every entry, where M N K <= 2^30.
The oracle's FP64 values are compared in FP32 for the every-entry check (torch CPU ops, all
cores): rounding C_ref and 1/D to FP32 moves the computed ratio by less than 1e-6, which is
taken off the tolerance.
"""
from __future__ import annotations

import numpy as np

from oracle import check

TOL = {0: 1e-5, 1: 8e-3}
FULL_LIMIT = 1 << 30
SAMPLE = 64          # rows and columns sampled per output (64 x 64 = 4,096 entries)
FP32_SLACK = 1e-6


def sample_index(seed: int, extent: int, n: int = SAMPLE) -> np.ndarray:
    """Sorted seeded indices in [0, extent): all of them if extent <= n."""
    if extent <= n:
        return np.arange(extent)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(extent, size=n, replace=False))


class Report:
    """Largest error ratio seen by each check, and counts."""

    def __init__(self, c_dtype: int):
        self.tol = TOL[c_dtype]
        self.frei = 0.0
        self.samp = 0.0
        self.full = 0.0
        self.zero_viol = 0
        self.outputs = 0
        self.full_outputs = 0
        self.worst = None

    def add(self, what, value, shape):
        if value > getattr(self, what):
            setattr(self, what, value)
            if value > (self.tol - FP32_SLACK if what == "full" else self.tol):
                self.worst = (what, value, shape)

    def ok(self) -> bool:
        return (self.frei <= self.tol and self.samp <= self.tol and self.full <= self.tol - FP32_SLACK
                and self.zero_viol == 0)

    def __str__(self):
        return ("%d outputs (%d every-entry): max Freivalds %.3e, sampled %.3e, every-entry %.3e, "
                "zero violations %d, tol %.0e%s" % (self.outputs, self.full_outputs, self.frei, self.samp,
                                                     self.full, self.zero_viol, self.tol,
                                                     "" if self.worst is None else ", worst %s" % (self.worst,)))


def device_reduce(torch, C, Xg, rows_g, cols_g):
    """On the device: C X (FP64) and the sampled block (FP32) of the M x N output C."""
    y = C.double() @ Xg[: C.shape[1]]
    s = C.index_select(0, rows_g).index_select(1, cols_g).float()
    return y, s


class FullRef:
    """FP64 C_ref and D of an output block, held as FP32 C_ref, FP32 1/D (0 where D = 0) and
    the D = 0 mask (torch CPU tensors) for every-entry comparisons of its leading rows."""

    def __init__(self, torch, c_ref, d):
        self.cr = torch.from_numpy(np.ascontiguousarray(c_ref, dtype=np.float32))
        dd = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float64))
        self.zero = dd == 0
        self.inv = torch.where(self.zero, torch.zeros_like(dd), 1.0 / dd).float()

    def ratio(self, torch, c_out, rows=None):
        """(max |C - C_ref| / D, zero violations) over the first `rows` rows (all by default);
        c_out a torch CPU tensor (BF16 or FP32) of that many rows."""
        m = c_out.shape[0] if rows is None else rows
        c = c_out.float()
        nz = int(torch.count_nonzero(self.zero[:m] & (c != 0)))
        r = float((c - self.cr[:m]).abs_().mul_(self.inv[:m]).max()) if c.numel() else 0.0
        return r, nz


def full_ratio(torch, c_out, c_ref, d):
    """Every-entry error ratio of an output (torch CPU tensor, BF16 or FP32) against FP64 C_ref
    and D (numpy), in FP32 on all cores; returns (ratio, zero violations)."""
    return FullRef(torch, c_ref, d).ratio(torch, c_out)


def check_one(torch, rep: Report, Af, Bf, X, y, rows, cols, samp, c_full=None, shape=None, Aabs=None, Babs=None):
    """All checks of one output from FP64 operand views Af (M x K), Bf (K x N): y = C X and
    samp = C[rows][:, cols] from the device, c_full the whole output (torch CPU) or None."""
    M, K = Af.shape
    N = Bf.shape[1]
    Aa = np.abs(Af) if Aabs is None else Aabs
    Ba = np.abs(Bf) if Babs is None else Babs
    rhs = Af @ (Bf @ X)
    bound = Aa @ (Ba @ np.abs(X))
    rep.add("frei", check.freivalds_ratio(y, rhs, bound, K, N), shape)
    Cb, Db = Af[rows] @ Bf[:, cols], Aa[rows] @ Ba[:, cols]
    e, zv = check.entries_ratio(samp, Cb, Db)
    rep.add("samp", e, shape)
    rep.zero_viol += zv
    if c_full is not None:
        Cr, D = check.reference_block(Af, Bf)
        e, zv = full_ratio(torch, c_full, Cr, D)
        rep.add("full", e, shape)
        rep.zero_viol += zv
        rep.full_outputs += 1
    rep.outputs += 1


def verify_landscape(torch, run, A_bits, B_bits, sizes, c_dtype, seed=17, log=print, device="cuda"):
    """Every (M, N, K) of the grid `sizes`^3 with operands viewed from pools (A: first M K
    elements as M x K, B: first K N as K x N).  run(M, N, K) runs the GEMM on the device and
    returns the output C (an M x N torch view, valid until the next call).  Host work is
    shared across the grid: B's rows do not depend on K and A's rows do not depend on M, so
    B X for the largest K serves every K, one product per K gives A (B X) for every M, and
    one sampled block per (K, N) serves every M."""
    rep = Report(c_dtype)
    maxd = int(sizes[-1])
    A64 = check.bf16_bits_to_f64(A_bits)
    B64 = check.bf16_bits_to_f64(B_bits)
    X = check.sign_vectors(seed, maxd, 2)
    Xg = torch.from_numpy(X).to(device)
    rows_of = {int(M): sample_index(seed * 7919 + int(M), int(M)) for M in sizes}
    cols_of = {int(N): sample_index(seed * 104729 + int(N), int(N)) for N in sizes}
    rows_g = {M: torch.from_numpy(r).to(device) for M, r in rows_of.items()}
    cols_g = {N: torch.from_numpy(c).to(device) for N, c in cols_of.items()}
    R_all = np.concatenate([rows_of[int(M)] for M in sizes])
    r_off = np.cumsum([0] + [rows_of[int(M)].size for M in sizes])
    BX, BXa = {}, {}
    for N in sizes:
        N = int(N)
        Bn = B64[: maxd * N].reshape(maxd, N)
        BX[N] = Bn @ X[:N]
        BXa[N] = np.abs(Bn) @ np.abs(X[:N])
    for K in sizes:
        K = int(K)
        # host side of this K that does not depend on the outputs
        A_K = A64[: maxd * K].reshape(maxd, K)
        A_Ka = np.abs(A_K)
        V = np.concatenate([BX[int(N)][:K] for N in sizes], axis=1)
        Va = np.concatenate([BXa[int(N)][:K] for N in sizes], axis=1)
        W, Wa = A_K @ V, A_Ka @ Va
        Ar, Ara = A_K[R_all], A_Ka[R_all]
        for j, N in enumerate(sizes):
            N = int(N)
            ys, ss, fulls = {}, {}, {}
            for M in sizes:
                M = int(M)
                C = run(M, N, K)
                ys[M], ss[M] = device_reduce(torch, C, Xg, rows_g[M], cols_g[N])
                if M * N * K <= FULL_LIMIT:
                    fulls[M] = C.cpu()
            if device == "cuda":
                torch.cuda.synchronize()
            B_KN = B64[: K * N].reshape(K, N)
            Bc = B_KN[:, cols_of[N]]
            blk, blka = Ar @ Bc, Ara @ np.abs(Bc)
            if fulls:
                ref = FullRef(torch, *check.reference_block(A_K[: max(fulls)], B_KN))
            for i, M in enumerate(sizes):
                M = int(M)
                y = ys[M].cpu().numpy()
                rep.add("frei", check.freivalds_ratio(y, W[:M, 2 * j:2 * j + 2], Wa[:M, 2 * j:2 * j + 2], K, N),
                        (M, N, K))
                a, b = r_off[i], r_off[i + 1]
                e, zv = check.entries_ratio(ss[M].cpu().numpy(), blk[a:b], blka[a:b])
                rep.add("samp", e, (M, N, K))
                rep.zero_viol += zv
                if M in fulls:
                    e, zv = ref.ratio(torch, fulls[M], M)
                    rep.add("full", e, (M, N, K))
                    rep.zero_viol += zv
                    rep.full_outputs += 1
                rep.outputs += 1
        log("K = %d done: %s" % (K, rep))
    return rep
