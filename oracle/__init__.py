"""CPU FP64 oracle for the PRTGS transfer path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The HIP library and its Python binding never import it,
and it never imports them; the only code the two sides share is the seeded
input generator module ``scenegen``.

The brute-force core is plain C (``prtgs_oracle.c``, compiled with gcc and
OpenMP, loaded with ctypes); relighting is an FP64 einsum and the gradients
are torch float64 autograd through a separate re-expression of the forward
(``oracle.grad``).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "prtgs_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# Default cutoffs: 3-sigma hit extent, peaks behind the origin ignored,
# transmittance below 1e-4 is opaque, no alpha floor, alpha clamped at 0.99.
# c_min: a ray is traced iff n . w > c_min; 0 as on the GPU path (other values
# only move the hemisphere threshold, to pin the deviation bound).
DEFAULT_CUT = dict(sigma_cut=3.0, t_min=0.0, T_eps=1e-4, alpha_min=0.0, alpha_max=0.99, c_min=0.0)
# Margins inside which an FP32 evaluation may resolve a predicate either way
# (the forms are in prtgs_oracle.c): |c| <= 1e-6; |d^2 - sigma_cut^2| <=
# 5e-5 (1 + kappa); |t* - t_min| <= 8e-5 (1 + d) / |W w| + 1e-5 |t*|;
# |T / T_eps - 1| <= 1e-4; two peak depths tied within the sum of their t*
# margins.  Each is at least 10x the largest error of a float32 model of the
# GPU's evaluation on the surface and million-splat workloads
# (tests/test_oracle_margins.py).
DEFAULT_MARGINS = (1e-6, 5e-5, 8e-5, 1e-4, 1e-5)


def build(force: bool = False) -> str:
    """Compile the C core with gcc (idempotent unless ``force``)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        build()
        lib = ctypes.CDLL(LIB)
        lib.ora_splitmix64.restype = ctypes.c_uint64
        lib.ora_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib_handle = lib
    return _lib_handle


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cut_array(cut):
    c = dict(DEFAULT_CUT)
    if cut:
        c.update(cut)
    return np.array([c["sigma_cut"], c["t_min"], c["T_eps"], c["alpha_min"], c["alpha_max"], c["c_min"]],
                    dtype=np.float64)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


# ----------------------------------------------------------------------------
# tables
# ----------------------------------------------------------------------------

def splitmix64(seed: int, index: int) -> int:
    return int(_lib().ora_splitmix64(ctypes.c_uint64(seed), ctypes.c_uint64(index)))


def grid(S: int):
    nu, nv = ctypes.c_int(), ctypes.c_int()
    _lib().ora_grid(ctypes.c_int(S), ctypes.byref(nu), ctypes.byref(nv))
    return nu.value, nv.value


def directions(S: int, seed: int = 0) -> np.ndarray:
    """[S,3] stratified directions (FP32 values held in FP64)."""
    out = np.empty((S, 3), dtype=np.float64)
    _lib().ora_directions(ctypes.c_int(S), ctypes.c_uint64(seed), _p(out))
    return out


def sh_basis(bands: int, dirs) -> np.ndarray:
    """[S, bands^2] real orthonormal SH at ``dirs`` (normalised inside)."""
    dirs = _f64(np.atleast_2d(dirs))
    K = bands * bands
    out = np.empty((dirs.shape[0], K), dtype=np.float64)
    lib = _lib()
    for s in range(dirs.shape[0]):
        row = np.ascontiguousarray(dirs[s])
        lib.ora_sh_basis(ctypes.c_int(bands), _p(row), out[s].ctypes.data_as(ctypes.c_void_p))
    return out


def tables(S: int, seed: int, bands: int):
    d = directions(S, seed)
    return d, sh_basis(bands, d)


# ----------------------------------------------------------------------------
# transfer
# ----------------------------------------------------------------------------

def _scene_arrays(scene):
    return (_f64(scene["means"]), _f64(scene["quats"]), _f64(scene["log_scales"]),
            _f64(scene["opacity"]), _f64(scene["normals"]))


def direct_transfer(scene, num_dirs, bands, seed=0, cut=None, sources=None, want_vis=False,
                    want_allow=False, margins=DEFAULT_MARGINS, threads=None, dirs=None, Y=None,
                    want_vis_bounds=False):
    """Direct (visibility) transfer t[count, K] of the listed sources.

    Returns dict(t=..., vis=[count,S] or None (-1 marks untraced rays),
    allow=[count,K] or None, vis_lo / vis_hi=[count,S] or None: the range
    of each ray's V over the other resolutions of its near-threshold
    predicates, -1 where the ray is not traced and its hemisphere test is
    not ambiguous).
    """
    means, quats, log_scales, opacity, normals = _scene_arrays(scene)
    n = means.shape[0]
    if dirs is None:
        dirs, Y = tables(num_dirs, seed, bands)
    K = Y.shape[1]
    src = np.arange(n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    count = src.shape[0]
    t = np.empty((count, K))
    vis = np.empty((count, num_dirs)) if want_vis else None
    allow = np.empty((count, K)) if want_allow else None
    vlo = np.empty((count, num_dirs)) if want_vis_bounds else None
    vhi = np.empty((count, num_dirs)) if want_vis_bounds else None
    mar = np.array(margins, dtype=np.float64) if (want_allow or margins is not None) else None
    _lib().ora_direct(ctypes.c_int(n), _p(means), _p(quats), _p(log_scales), _p(opacity), _p(normals),
                      ctypes.c_int(num_dirs), _p(_f64(dirs)), ctypes.c_int(K), _p(_f64(Y)),
                      _p(_cut_array(cut)), _p(mar), _p(src), ctypes.c_int(count), _p(t), _p(vis),
                      _p(allow), _p(vlo), _p(vhi), ctypes.c_int(threads or default_threads()))
    return dict(t=t, vis=vis, allow=allow, vis_lo=vlo, vis_hi=vhi)


def hit_set(scene, num_dirs, seed=0, cut=None, sources=None, margins=DEFAULT_MARGINS, threads=None):
    """Sorted indices of every Gaussian hit by a traced ray of ``sources``."""
    means, quats, log_scales, opacity, normals = _scene_arrays(scene)
    n = means.shape[0]
    dirs = directions(num_dirs, seed)
    src = np.arange(n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    mark = np.zeros(n, dtype=np.uint8)
    _lib().ora_hit_set(ctypes.c_int(n), _p(means), _p(quats), _p(log_scales), _p(opacity), _p(normals),
                       ctypes.c_int(num_dirs), _p(dirs), _p(_cut_array(cut)),
                       _p(np.array(margins, dtype=np.float64)), _p(src), ctypes.c_int(src.shape[0]),
                       _p(mark), ctypes.c_int(threads or default_threads()))
    return np.nonzero(mark)[0].astype(np.int64)


def rays_vis(scene, sources, dirs, cut=None, threads=None):
    """Visibility V[r] of the ray from the centre of Gaussian sources[r]
    along dirs[r] (unit), through every other Gaussian."""
    means, quats, log_scales, opacity, _ = _scene_arrays(scene)
    n = means.shape[0]
    src = np.ascontiguousarray(sources, dtype=np.int32)
    w = _f64(dirs).reshape(-1, 3)
    V = np.empty(src.shape[0])
    _lib().ora_rays_vis(ctypes.c_int(n), _p(means), _p(quats), _p(log_scales), _p(opacity),
                        ctypes.c_int(src.shape[0]), _p(src), _p(w), _p(_cut_array(cut)), _p(V),
                        ctypes.c_int(threads or default_threads()))
    return V


def bounce_transfer(scene, num_dirs, bands, t_dir_rows, t_dir_index, allow_dir_rows=None, seed=0,
                    cut=None, sources=None, want_allow=False, margins=DEFAULT_MARGINS, threads=None):
    """One-bounce indirect transfer t_ind[count, 3, K] of the listed sources.

    ``t_dir_rows[r]`` is the direct transfer of Gaussian ``t_dir_index[r]``
    (every Gaussian hit by a traced ray of the sources must be listed).
    """
    means, quats, log_scales, opacity, normals = _scene_arrays(scene)
    albedo = _f64(scene["albedo"])
    n = means.shape[0]
    dirs, Y = tables(num_dirs, seed, bands)
    K = Y.shape[1]
    slot = np.full(n, -1, dtype=np.int32)
    slot[np.asarray(t_dir_index)] = np.arange(len(t_dir_index), dtype=np.int32)
    src = np.arange(n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    count = src.shape[0]
    out = np.empty((count, 3, K))
    allow = np.empty((count, 3, K)) if want_allow else None
    rows = _f64(t_dir_rows)
    arows = _f64(allow_dir_rows) if allow_dir_rows is not None else None
    mar = np.array(margins, dtype=np.float64)
    missing = _lib().ora_bounce(ctypes.c_int(n), _p(means), _p(quats), _p(log_scales), _p(opacity),
                                _p(normals), _p(albedo), ctypes.c_int(num_dirs), _p(dirs), ctypes.c_int(K),
                                _p(_cut_array(cut)), _p(mar), _p(slot), _p(rows), _p(arows), _p(src),
                                ctypes.c_int(count), _p(out), _p(allow),
                                ctypes.c_int(threads or default_threads()))
    if missing:
        raise ValueError("a hit Gaussian has no direct transfer row")
    return dict(t=out, allow=allow)


def full_transfer(scene, num_dirs, bands, bounces, seed=0, cut=None, sources=None, want_allow=False,
                  margins=DEFAULT_MARGINS, threads=None):
    """Transfer of the listed sources: [count, 1, K] (direct) or [count, 3, K]
    (direct in every channel plus the one-bounce term)."""
    n = scene["means"].shape[0]
    src = np.arange(n) if sources is None else np.asarray(sources)
    d = direct_transfer(scene, num_dirs, bands, seed, cut, src, want_allow=want_allow, margins=margins,
                        threads=threads)
    if bounces == 0:
        return dict(t=d["t"][:, None, :], allow=None if d["allow"] is None else d["allow"][:, None, :])
    need = hit_set(scene, num_dirs, seed, cut, src, margins, threads)
    dj = direct_transfer(scene, num_dirs, bands, seed, cut, need, want_allow=True, margins=margins,
                         threads=threads)
    b = bounce_transfer(scene, num_dirs, bands, dj["t"], need, dj["allow"], seed, cut, src,
                        want_allow=want_allow, margins=margins, threads=threads)
    t = d["t"][:, None, :] + b["t"]
    allow = None
    if want_allow:
        allow = d["allow"][:, None, :] + b["allow"]
    return dict(t=t, allow=allow, t_dir=d["t"], t_ind=b["t"])


# ----------------------------------------------------------------------------
# the paper's own bounce: index matrix + recursive self-transfer
# (Sec. 4.4 Eq. 26 and the filter after Eq. 27; Sec. 4.5 Eq. 32-35)
# ----------------------------------------------------------------------------

def index_matrix(scene, num_dirs, seed=0, cut=None, t_same=1.0, sources=None, margins=DEFAULT_MARGINS,
                 threads=None):
    """idx[count, S]: per ray the hit of largest W = alpha T max(-w.n_j, 0)
    among hits with T <= t_same (-1: none, or not traced); amb[count, S]:
    rays whose choice lies within FP32 rounding of a tie or threshold."""
    means, quats, log_scales, opacity, normals = _scene_arrays(scene)
    n = means.shape[0]
    dirs = directions(num_dirs, seed)
    src = np.arange(n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    idx = np.empty((src.shape[0], num_dirs), dtype=np.int32)
    amb = np.empty((src.shape[0], num_dirs), dtype=np.uint8)
    mar = None if margins is None else np.array(margins, dtype=np.float64)
    _lib().ora_index(ctypes.c_int(n), _p(means), _p(quats), _p(log_scales), _p(opacity), _p(normals),
                     ctypes.c_int(num_dirs), _p(dirs), _p(_cut_array(cut)), ctypes.c_double(t_same), _p(mar),
                     _p(src), ctypes.c_int(src.shape[0]), _p(idx), _p(amb), ctypes.c_int(threads or default_threads()))
    return idx, amb.astype(bool)


def self_transfer(scene, num_dirs, index, t_prev, seed=0, sources=None):
    """One recursion step of the self-transfer (Eq. 32-34):
    t[q, c, :] = (4 pi / S) sum_{s: idx >= 0} max(0, n_i . w_s) (rho_{j,c} / pi) t_prev[j, c', :]
    with i = sources[q], j = index[q, s], c' = c for an RGB t_prev [n, 3, K] and
    0 for a mono one [n, 1, K].  FP64."""
    normals = _f64(scene["normals"])
    albedo = _f64(scene["albedo"])
    tp = _f64(t_prev)
    n = normals.shape[0]
    src = np.arange(n) if sources is None else np.asarray(sources)
    dirs = directions(num_dirs, seed)
    S = dirs.shape[0]
    out = np.zeros((len(src), 3, tp.shape[2]))
    for q, i in enumerate(src):
        c = normals[i] @ dirs.T
        for s in range(S):
            j = int(index[q, s])
            if j < 0 or not c[s] > 0.0:
                continue
            for ch in range(3):
                out[q, ch] += (4.0 * math.pi / S) * c[s] * albedo[j, ch] / math.pi * tp[j, ch if tp.shape[1] == 3 else 0]
    return out


def index_transfer(scene, num_dirs, bands, bounces, seed=0, cut=None, t_same=1.0, threads=None):
    """Total transfer of every splat with the paper's bounce (Eq. 35 with the
    direct term, reading c14): sum_{m=0..bounces} T^m, T^0 the direct
    transfer, T^m = self_transfer(T^{m-1}).  Returns dict(t=[n,3,K] (or
    [n,1,K] for bounces = 0), index, amb, terms=[T^0, ..., T^bounces])."""
    n = scene["means"].shape[0]
    d = direct_transfer(scene, num_dirs, bands, seed, cut, threads=threads)["t"][:, None, :]
    terms = [d]
    if bounces == 0:
        return dict(t=d, index=None, amb=None, terms=terms)
    idx, amb = index_matrix(scene, num_dirs, seed, cut, t_same, threads=threads)
    total = np.repeat(d, 3, axis=1)
    prev = d
    for _ in range(bounces):
        prev = self_transfer(scene, num_dirs, idx, prev, seed)
        terms.append(prev)
        total = total + prev
    return dict(t=total, index=idx, amb=amb, terms=terms)


# ----------------------------------------------------------------------------
# relighting (Eq. 14: rendering reduces to a dot product in the SH domain)
# ----------------------------------------------------------------------------

def relight(transfer, light):
    """colour[n, b, c] = sum_k T[n, c', k] L[b, c, k], c' = c for RGB transfer,
    0 for a single-channel one.  FP64."""
    T = np.asarray(transfer, dtype=np.float64)
    L = np.asarray(light, dtype=np.float64)
    if T.ndim == 2:
        T = T[:, None, :]
    if T.shape[1] == 1:
        return np.einsum("nk,bck->nbc", T[:, 0, :], L)
    return np.einsum("nck,bck->nbc", T, L)


def relight_grads(transfer, light, d_colour):
    """Gradients of sum(d_colour * relight(transfer, light)) with respect to
    transfer and light, by torch float64 autograd of the dot product."""
    import torch
    T = torch.tensor(np.asarray(transfer, dtype=np.float64), requires_grad=True)
    L = torch.tensor(np.asarray(light, dtype=np.float64), requires_grad=True)
    dC = torch.from_numpy(np.asarray(d_colour, dtype=np.float64))
    if T.shape[1] == 1:
        C = torch.einsum("nk,bck->nbc", T[:, 0, :], L)
    else:
        C = torch.einsum("nck,bck->nbc", T, L)
    (C * dC).sum().backward()
    return T.grad.numpy(), L.grad.numpy()
