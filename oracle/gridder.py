"""Convolutional gridding and degridding with separable or exact GCF tables (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2 (W projection equation): the dirty image is F^-1 of the sum over
visibilities of W_i V_i convolved with the GCF for w_i.  Section 5: with the
separable GCF  F~_w(u, v) = F1_w(u) F1_w(v)  the update of grid cell (u, v) by
visibility i is  W_i V_i F1(u - u_i) F1(v - v_i),  and the partial product
W_i V_i F1(u - u_i) is formed once per column and reused for every row.

Gridding (visibility i with bins cu, fu, cv, fv, k and h = floor(S/2)):
    r[s] = W_i V_i Tu[k][fu][s]                          (row product)
    G[cv - h + t][cu - h + s] += r[s] * Tv[k][fv][t]     s, t in [0, S)
Degridding is its adjoint:
    V_i = sum_t conj(Tv[k][fv][t]) sum_s conj(Tu[k][fu][s]) G[cv-h+t][cu-h+s].
Tu and Tv are the same table in plain mode and the facet l / m tables in
Section 4.1's facet mode.

``wrap=True`` indexes cells modulo N; it exists only for the full-support pins
(S = N), never for the product path, which drops off-grid footprints.
"""
import numpy as np


def _footprint_index(q, N, S, wrap):
    h = S // 2
    s = np.arange(S)
    ju = q['cell_u'][:, None] - h + s[None, :]      # [n][S]
    jv = q['cell_v'][:, None] - h + s[None, :]      # [n][S]
    if wrap:
        ju, jv = ju % N, jv % N
    return ju, jv


def _kept(q):
    return np.flatnonzero(~q['dropped'])


def grid_separable(q, y, Tu, N, S, Tv=None, wrap=False, chunk=20000):
    """G[jv][ju] (complex128 N x N) = sum over kept visibilities of the
    separable footprint y_i Tu[...][s] Tv[...][t]."""
    if Tv is None:
        Tv = Tu
    G = np.zeros(N * N, dtype=np.complex128)
    idx = _kept(q)
    for c0 in range(0, len(idx), chunk):
        sel = idx[c0:c0 + chunk]
        qs = {key: val[sel] for key, val in q.items()}
        ju, jv = _footprint_index(qs, N, S, wrap)
        tu = Tu[qs['k'], qs['fi_u']]                 # [n][S]
        tv = Tv[qs['k'], qs['fi_v']]                 # [n][S]
        r = y[sel][:, None] * tu                     # row product
        contrib = tv[:, :, None] * r[:, None, :]     # [n][t][s]
        flat = (jv[:, :, None] * N + ju[:, None, :]).ravel()
        G += np.bincount(flat, weights=contrib.real.ravel(), minlength=N * N)
        G += 1j * np.bincount(flat, weights=contrib.imag.ravel(), minlength=N * N)
    return G.reshape(N, N)


def degrid_separable(q, G, Tu, N, S, Tv=None, wrap=False, chunk=20000):
    """V_i (complex128); zero for dropped visibilities."""
    if Tv is None:
        Tv = Tu
    n = len(q['dropped'])
    V = np.zeros(n, dtype=np.complex128)
    idx = _kept(q)
    for c0 in range(0, len(idx), chunk):
        sel = idx[c0:c0 + chunk]
        qs = {key: val[sel] for key, val in q.items()}
        ju, jv = _footprint_index(qs, N, S, wrap)
        tu = np.conj(Tu[qs['k'], qs['fi_u']])
        tv = np.conj(Tv[qs['k'], qs['fi_v']])
        patch = G[jv[:, :, None], ju[:, None, :]]    # [n][t][s]
        inner = np.einsum('nts,ns->nt', patch, tu)
        V[sel] = np.einsum('nt,nt->n', inner, tv)
    return V


def grid_exact(q, y, T2, N, S, wrap=False):
    """Gridding with the non-separable table T2[k][fu][fv][su][sv]."""
    G = np.zeros(N * N, dtype=np.complex128)
    idx = _kept(q)
    qs = {key: val[idx] for key, val in q.items()}
    ju, jv = _footprint_index(qs, N, S, wrap)
    ker = T2[qs['k'], qs['fi_u'], qs['fi_v']]       # [n][su][sv]
    contrib = y[idx][:, None, None] * np.transpose(ker, (0, 2, 1))  # [n][sv][su]
    flat = (jv[:, :, None] * N + ju[:, None, :]).ravel()
    G += np.bincount(flat, weights=contrib.real.ravel(), minlength=N * N)
    G += 1j * np.bincount(flat, weights=contrib.imag.ravel(), minlength=N * N)
    return G.reshape(N, N)


def degrid_exact(q, G, T2, N, S, wrap=False):
    n = len(q['dropped'])
    V = np.zeros(n, dtype=np.complex128)
    idx = _kept(q)
    qs = {key: val[idx] for key, val in q.items()}
    ju, jv = _footprint_index(qs, N, S, wrap)
    ker = np.conj(T2[qs['k'], qs['fi_u'], qs['fi_v']])  # [n][su][sv]
    patch = G[jv[:, :, None], ju[:, None, :]]           # [n][sv][su]
    V[idx] = np.einsum('nvu,nuv->n', patch, ker)
    return V


def grid_cells(q, y, Tu, N, S, cells, Tv=None):
    """Selected grid cells only: G[jv][ju] for each (jv, ju) in ``cells``,
    summing over every kept visibility whose footprint covers the cell.  Used
    to check full-size gridding at sampled outputs."""
    if Tv is None:
        Tv = Tu
    h = S // 2
    keep = ~q['dropped']
    out = np.zeros(len(cells), dtype=np.complex128)
    for n, (jv, ju) in enumerate(cells):
        s = ju - q['cell_u'] + h
        t = jv - q['cell_v'] + h
        m = keep & (s >= 0) & (s < S) & (t >= 0) & (t < S)
        i = np.flatnonzero(m)
        out[n] = np.sum(y[i] * Tu[q['k'][i], q['fi_u'][i], s[i]] * Tv[q['k'][i], q['fi_v'][i], t[i]])
    return out
