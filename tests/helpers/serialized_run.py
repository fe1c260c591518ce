"""Digest of a fixed set of outputs of every GPU path (plain, batched,
streamed, served), printed as one hex line. Run once normally and once with
the ROCm runtime serialising kernels and copies: the digests must agree,
i.e. no result depends on how the streams' work interleaves."""
import hashlib
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_1609_01257_amd import inputs, rngx  # noqa: E402


def digest() -> str:
    h = hashlib.sha256()
    rngx.init(12345, 65537)
    out = torch.empty(5 * 65537, dtype=torch.int64, device="cuda")
    rngx.generate(5, out)
    torch.cuda.synchronize()
    h.update(out.cpu().numpy().tobytes())

    r = inputs.ragged_requests(m=31, seed=4, max_len=100000, max_offset=10**6)
    reqs = rngx.make_reqs(r.seeds, r.gids, r.offsets, r.lengths)
    bout = torch.empty(r.total, dtype=torch.int64, device="cuda")
    for per_item in (False, True):
        rngx.set_batch_cfg(128, 4, 0, True, 16, 1, per_item)
        rngx.generate_batch(reqs, bout)
        torch.cuda.synchronize()
        h.update(bout.cpu().numpy().tobytes())

    rngx.init(42, 4099)
    dev0 = torch.empty(4099, dtype=torch.int64, device="cuda")
    dev1 = torch.empty(4099, dtype=torch.int64, device="cuda")
    host = torch.zeros(6 * 4099, dtype=torch.int64, pin_memory=True)
    rngx.stream_to_host(6, 1, dev0, dev1, host, 6)
    h.update(host.numpy().tobytes())

    pool = torch.zeros(32 << 20, dtype=torch.uint8, device="cuda")
    rngx.serve_start(9, 64, pool, 4, 8)
    tickets = [rngx.serve_submit(g % 64, 1000 + 97 * g) for g in range(40)]
    for g, t in enumerate(tickets):
        ptr = rngx.serve_wait(t, 30.0)
        off = ptr - pool.data_ptr()
        n = 1000 + 97 * g
        h.update(pool[off:off + 8 * n].cpu().numpy().tobytes())
        rngx.serve_release(t)
    rngx.serve_stop()
    rngx.shutdown()
    return h.hexdigest()


if __name__ == "__main__":
    print(digest(), flush=True)
