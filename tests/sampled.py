"""Oracle reference for sampled k-points of a full-size history pass: the stored blocks of one
k are read back from the device history in its packed layout (include/kbe.h) and handed to the
oracle as a one-k system (the history sums are independent per k)."""
import numpy as np

from oracle import oracle as O


def collision_reference(K, S, cfg, m, k, sig_all):
    """I(t_m, .) of k-point ``k`` from the oracle, given the device history of System ``S`` and
    the Sigma row ``sig_all`` ([t_j][k][2][nb][nb], as ``S.sigma_row(m)`` returns it)."""
    nb = cfg.nb
    C = 2 * nb * nb
    hk = S.history_blocks()[k].cpu().numpy().astype(np.complex128)  # [C * P]
    rows = []
    for j in range(m + 1):
        c, tp = np.meshgrid(np.arange(C), np.arange(j + 1), indexing="ij")
        blk = hk[K.hist_offset(c, j, tp, S.nt_max, C, S.fp32, S.mfma)]  # [C][t']
        rows.append(blk.T.reshape(j + 1, 1, 2, nb, nb))
    return O.collision_row(cfg.replace(nkx=1, nky=1), m, rows, sig_all[:, k:k + 1])
