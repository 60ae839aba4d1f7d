"""Reference computation of the 32 bracket-network inputs of a mixed cell
(TEST INFRASTRUCTURE ONLY; the HIP library computes the same quantities on
its own).

Per mixed cell P, with phi the vertex field, W = phi_max - phi_min, the face
unit normals n_f (out of P) and areas A_f, and alpha_Q the face neighbours'
fractions (alpha_P on boundary faces):

  0      alpha_P
  1-7    (q-quantile of the cell's vertex values - phi_min)/W, q = 1/8..7/8,
         linear between order statistics: t = q (nv-1), i = floor(t)
  8      (mean vertex value - phi_min)/W
  9      W
  10-12  sum_f A_f (alpha_Q - alpha_P) n_f / sum_f A_f
  13-18  sum_f A_f (alpha_Q - alpha_P) n_f n_f^T / sum_f A_f   (xx yy zz xy xz yz)
  19-24  sum_f A_f n_f n_f^T / sum_f A_f                       (xx yy zz xy xz yz)
  25     number of faces / 32
  26-28  mean, min, max of alpha_Q over interior neighbours (alpha_P if none)
  29-31  0

Targets: u* = (s* - phi_min)/W and the interface normal n*.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 32


def cell_features(mesh, geom, phi, alpha, cells) -> tuple[np.ndarray, np.ndarray]:
    """Features [len(cells), 32] (float64) and (phi_min, W) [len(cells), 2]."""
    out = np.zeros((len(cells), N_FEAT))
    rng = np.zeros((len(cells), 2))
    Sf = geom.Sf
    for r, P in enumerate(cells):
        faces = mesh.cell_face[mesh.cell_face_off[P]:mesh.cell_face_off[P + 1]]
        vids = np.unique(np.concatenate([mesh.face_vert[mesh.face_vert_off[f]:mesh.face_vert_off[f + 1]]
                                         for f in faces]))
        v = np.sort(phi[vids])
        pmin, pmax = v[0], v[-1]
        W = pmax - pmin
        rng[r] = (pmin, W)
        aP = alpha[P]
        out[r, 0] = aP
        nv = len(v)
        for qi in range(7):
            q = (qi + 1) / 8.0
            t = q * (nv - 1)
            i = int(np.floor(t))
            fr = t - i
            val = v[i] if i + 1 >= nv else v[i] + fr * (v[i + 1] - v[i])
            out[r, 1 + qi] = (val - pmin) / W if W > 0 else 0.0
        out[r, 8] = (v.mean() - pmin) / W if W > 0 else 0.0
        out[r, 9] = W
        Atot = 0.0
        m1 = np.zeros(3)
        m2 = np.zeros(6)
        sh = np.zeros(6)
        nb = []
        for f in faces:
            S = Sf[:, f] * (1.0 if mesh.face_owner[f] == P else -1.0)
            A = np.linalg.norm(S)
            n = S / A
            Q = mesh.face_neigh[f] if mesh.face_owner[f] == P else mesh.face_owner[f]
            aQ = alpha[Q] if Q >= 0 else aP
            if Q >= 0:
                nb.append(alpha[Q])
            da = aQ - aP
            outer = np.array([n[0] * n[0], n[1] * n[1], n[2] * n[2], n[0] * n[1], n[0] * n[2], n[1] * n[2]])
            m1 += A * da * n
            m2 += A * da * outer
            sh += A * outer
            Atot += A
        out[r, 10:13] = m1 / Atot
        out[r, 13:19] = m2 / Atot
        out[r, 19:25] = sh / Atot
        out[r, 25] = len(faces) / 32.0
        if nb:
            out[r, 26:29] = (np.mean(nb), np.min(nb), np.max(nb))
        else:
            out[r, 26:29] = aP
    return out, rng
