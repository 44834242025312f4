"""Test helpers: run the oracle on (a sample of) a synthetic problem, compare bitwise."""
import numpy as np

from oracle import codec, spmv as ospmv


def decode_vec(h, idx=None):
    """Oracle-side decode of a host MP array (optionally only the entries in idx)."""
    if idx is None:
        return codec.decode(h.limbs, h.hdr, h.p)
    idx = np.asarray(idx, dtype=np.int64)
    vals = codec.decode(h.limbs[:, idx], h.hdr[idx], h.p)
    return dict(zip(idx.tolist(), vals))


def oracle_spmv_rows(A, x, rows, mode):
    """Oracle y_i for the given rows of host CSR A and host vector x."""
    rows = np.asarray(rows, dtype=np.int64)
    rp = A.row_ptr.astype(np.int64)
    sub_rp = [0]
    ks = []
    for i in rows:
        ks.extend(range(int(rp[i]), int(rp[i + 1])))
        sub_rp.append(len(ks))
    ks = np.asarray(ks, dtype=np.int64)
    cols = A.col_idx[ks] if len(ks) else np.zeros(0, np.int32)
    vals = codec.decode(A.vals.limbs[:, ks], A.vals.hdr[ks], A.vals.p) if len(ks) else []
    xs = decode_vec(x, np.unique(cols)) if len(ks) else {}
    return ospmv.spmv(sub_rp, cols.tolist(), vals, xs, A.vals.p, mode)


def encode(vals, p):
    return codec.encode(vals, p)


def assert_bitwise(gpu_limbs, gpu_hdr, want_vals, p, rows=None, what=""):
    """The GPU's (limbs, hdr) at `rows` equal the oracle's values bit for bit."""
    wl, wh = codec.encode(want_vals, p)
    if rows is not None:
        gpu_limbs = gpu_limbs[:, rows]
        gpu_hdr = gpu_hdr[rows]
    bad = np.nonzero((gpu_hdr != wh) | np.any(gpu_limbs != wl, axis=0))[0]
    if len(bad):
        i = int(bad[0])
        got = codec.decode(gpu_limbs[:, i:i + 1], gpu_hdr[i:i + 1], p)[0]
        raise AssertionError("%s: %d of %d differ; first at %d: gpu %r oracle %r"
                             % (what, len(bad), len(wh), i if rows is None else int(np.asarray(rows)[i]),
                                got, want_vals[i]))


def digest(limbs, hdr):
    """SHA-256 of an MP array in the storage layout (limb planes, then headers, little endian):
    the form in which the stored expected values of long runs are compared."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.asarray(limbs, dtype="<u4")).tobytes())
    h.update(np.ascontiguousarray(np.asarray(hdr, dtype="<i4")).tobytes())
    return h.hexdigest()
