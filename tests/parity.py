"""Helpers shared by the GPU parity tests: device copies of the seeded
inputs, device-side ordering of large record sets, and the element-by-element
comparison with the oracle (result sets identical, endpoints within 1e-9
relative)."""
import numpy as np

import oracle

REL = 1e-9
RESULT_DTYPE = oracle.RESULT_DTYPE


def device_segments(S):
    """The segment arrays of S as contiguous CUDA tensors (float64, int32 traj)."""
    import torch
    out = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda()
           for k, v in S.arrays().items() if k != "traj"}
    out["traj"] = torch.from_numpy(np.ascontiguousarray(S.traj).astype(np.int32)).cuda()
    return out


def compare(got, want, label=""):
    """Records of the GPU against the oracle's: the same (q_seg, e_seg) pairs
    with the same trajectory ids and no duplicates, endpoints within REL
    relative.  Both must be in (q_seg, e_seg) order.  Returns the number of
    records whose endpoints are bit-identical."""
    kg = got["q_seg"].astype(np.uint64) << np.uint64(32) | got["e_seg"]
    assert np.all(kg[1:] > kg[:-1]), f"{label}: records not unique or not in key order"
    assert got.size == want.size, f"{label}: {got.size} records, oracle {want.size}"
    for f in ("q_seg", "e_seg", "q_traj", "e_traj"):
        assert np.array_equal(got[f], want[f]), f"{label}: field {f} differs"
    for f in ("t_lo", "t_hi"):
        err = np.abs(got[f] - want[f])
        tol = REL * np.maximum(1.0, np.abs(want[f]))
        assert np.all(err <= tol), f"{label}: {f} max err {err.max()}"
    return int(np.sum((got["t_lo"] == want["t_lo"]) & (got["t_hi"] == want["t_hi"])))


class DeviceRecords:
    """n result records in a CUDA byte tensor, ordered on the device by
    (q_seg, e_seg) so that slices by query segment can be taken to the host a
    piece at a time (the full set of a large search does not need to be held
    on the host at once)."""

    def __init__(self, buf, n):
        import torch
        self.n = n
        rec = buf[: n * 32].view(torch.int64).view(n, 4)
        ids = rec[:, 0]
        q = ids & 0xFFFFFFFF
        e = (ids >> 32) & 0xFFFFFFFF
        key = (q << 32) | e
        self.key, perm = torch.sort(key)
        self.rec = rec[perm]
        del perm, key
        self.unique = bool((self.key[1:] > self.key[:-1]).all().item()) if n > 1 else True

    def q_range(self, q0, q1):
        """Records with q0 <= q_seg < q1, as a host array in key order."""
        import torch
        bounds = torch.tensor([q0 << 32, q1 << 32], dtype=torch.int64, device=self.key.device)
        a, b = torch.searchsorted(self.key, bounds).tolist()
        host = self.rec[a:b].cpu().numpy()
        return np.frombuffer(host.tobytes(), dtype=RESULT_DTYPE).copy()

    def equal(self, other):
        """Bitwise equality of two ordered record sets."""
        import torch
        return self.n == other.n and bool(torch.equal(self.rec, other.rec))
