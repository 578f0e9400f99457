"""Helpers for the CPU tests of the library's host logic (no GPU calls)."""
import ctypes

import numpy as np

from paper_2205_04194_amd import _lib


def host_tree(xy_list, c_list, leaf, p=4, max_level=0, level_order=None, direct_max=0):
    """Build the host part of a tree; returns (handle, status)."""
    lib = _lib.load()
    xy = np.concatenate(xy_list, axis=0)
    offs = np.concatenate([[0], np.cumsum([len(a) for a in xy_list])]).astype(np.int64)
    x = np.ascontiguousarray(xy[:, 0], dtype=np.float64)
    y = np.ascontiguousarray(xy[:, 1], dtype=np.float64)
    c = np.ascontiguousarray(c_list, dtype=np.float64)
    prm = _lib.params(leaf, p, max_level, level_order, direct_max)
    st = ctypes.c_int(0)
    dp = ctypes.POINTER(ctypes.c_double)
    h = lib.imq_debug_host_tree(len(xy_list), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                x.ctypes.data_as(dp), y.ctypes.data_as(dp), c.ctypes.data_as(dp),
                                ctypes.byref(prm), ctypes.byref(st))
    return h, st.value


_DTYPES = {"xl": np.float64, "yl": np.float64, "cx": np.float64, "cy": np.float64,
           "side": np.float64, "cn": np.float64, "pt_scale": np.float64, "lox": np.float64,
           "loy": np.float64}

FIELDS = ["perm", "xl", "yl", "pt_scale", "pt_leaf", "level", "set", "ix", "iy", "parent", "child0",
          "nchild", "pos", "begin", "end", "isleaf", "cx", "cy", "level_begin", "leaves", "u_off", "u_idx",
          "v_off", "v_idx", "v_cls", "w_off", "w_idx", "x_off", "x_idx", "Klev", "side", "lox", "loy", "cn",
          "sh_par", "sh_kids", "sh_level_begin", "near_expand"]


def device_tree(xy_list, c_list, leaf, p=4, max_level=0, level_order=None, direct_max=0):
    """The same tree from the device construction (needs a GPU); returns (handle, status)."""
    lib = _lib.load()
    xy = np.concatenate(xy_list, axis=0)
    offs = np.concatenate([[0], np.cumsum([len(a) for a in xy_list])]).astype(np.int64)
    x = np.ascontiguousarray(xy[:, 0], dtype=np.float64)
    y = np.ascontiguousarray(xy[:, 1], dtype=np.float64)
    c = np.ascontiguousarray(c_list, dtype=np.float64)
    prm = _lib.params(leaf, p, max_level, level_order, direct_max)
    st = ctypes.c_int(0)
    dp = ctypes.POINTER(ctypes.c_double)
    h = lib.imq_debug_device_tree(len(xy_list), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  x.ctypes.data_as(dp), y.ctypes.data_as(dp), c.ctypes.data_as(dp),
                                  ctypes.byref(prm), ctypes.byref(st))
    return h, st.value


def get(h, name):
    lib = _lib.load()
    n = lib.imq_debug_host_tree_size(h, name.encode())
    assert n >= 0, name
    out = np.empty(n, dtype=_DTYPES.get(name, np.int32))
    assert lib.imq_debug_host_tree_get(h, name.encode(), out.ctypes.data_as(ctypes.c_void_p)) == 0
    return out


def free(h):
    _lib.load().imq_debug_host_tree_free(h)


def table(kind, p, pos=0, level=0, dx=0, dy=0, cnorm=0.0):
    K = (p + 1) * (p + 2) // 2
    out = np.zeros(K if kind == 3 else K * K)
    rc = _lib.load().imq_debug_table(kind, p, pos, level, dx, dy, cnorm,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0
    return out if kind == 3 else out.reshape(K, K)


# ---- the stored representation, written from its definition -----------------
# coefficient layout: degree n = 0..p, m ascending with n+m even, (Re, Im)

def layout(p):
    lay = []
    for n in range(p + 1):
        for m in range(n % 2, n + 1, 2):
            lay.append((n, m, 0))
            if m > 0:
                lay.append((n, m, 1))
    return lay


def moments(p, pts, u, z, s):
    """Mt[n,m] = sum u |w|^(n-m) conj(w)^m, w = (y - z)/s."""
    w = ((pts[:, 0] - z[0]) + 1j * (pts[:, 1] - z[1])) / s
    out = []
    for n, m, ri in layout(p):
        v = np.sum(u * np.abs(w) ** (n - m) * np.conj(w) ** m)
        out.append(v.real if ri == 0 else v.imag)
    return np.array(out)


def local_eval(p, Lt, pts, z, s):
    """sum Re(Lt[n,m] |w|^(n-m) w^m), w = (x - z)/s."""
    w = ((pts[:, 0] - z[0]) + 1j * (pts[:, 1] - z[1])) / s
    phi = np.zeros(len(pts))
    lay = layout(p)
    for i, (n, m, ri) in enumerate(lay):
        mono = np.abs(w) ** (n - m) * w ** m
        phi += Lt[i] * (mono.real if ri == 0 else -mono.imag)
    return phi


def odd_layout(p):
    """n+m-odd local coefficients (j >= 1, k = j-1, j-3, ... >= 0), (Re, Im)."""
    lay = []
    for j in range(1, p + 1):
        for k in range((j + 1) % 2, j, 2):
            lay.append((j, k, 0))
            if k > 0:
                lay.append((j, k, 1))
    return lay


def vertical_eval(p, Lo, pts, z, s):
    """sum Re(Lo[j,k] |w|^(j-1-k) w^k), w = (x - z)/s: the z-derivative at the plane."""
    w = ((pts[:, 0] - z[0]) + 1j * (pts[:, 1] - z[1])) / s
    out = np.zeros(len(pts))
    for i, (j, k, ri) in enumerate(odd_layout(p)):
        mono = np.abs(w) ** (j - 1 - k) * w ** k
        out += Lo[i] * (mono.real if ri == 0 else -mono.imag)
    return out
