"""End-to-end two-server PIR on one GPU (IM-PIR Sec. 2-3, Algorithm 1).

A client and two non-colluding servers that each hold a replica of the
database.  For every record it wants, the client generates a pair of DPF keys
(Sec. 3.1), sends one key to each server, and XORs the two answers (the
client step of Algorithm 1).  Each server evaluates its key over the whole
domain on the GPU and scans its replica (Sec. 3.2-3.3); neither key alone
says anything about the index.  Midway the database owner pushes the same
record update to both servers; each applies it in an idle window of its
request stream (Sec. 3.3), so every query is answered from one whole version.

Both "servers" run on the same GPU here (two contexts, two resident
replicas); over a network they would be two machines.

    python -m paper_2509_06514_amd.two_server [--records N] [--record-bytes R] [--queries Q]
"""
import argparse
import json
import secrets
import time

import numpy as np

from . import Context, Server, dpf_domain_bits, dpf_gen, reconstruct
from ._native import PIR_OK


def _fetch(servers, db_ids, n_bits, indices, record_bytes):
    """Client: one key pair per index, submitted to both servers, answers reconstructed."""
    outs = [np.zeros((len(indices), record_bytes), np.uint8) for _ in servers]
    tickets = [[] for _ in servers]
    for q, i in enumerate(indices):
        k0, k1 = dpf_gen(int(i), n_bits, secrets.token_bytes(16), secrets.token_bytes(16))
        for s, (srv, key) in enumerate(zip(servers, (k0, k1))):
            tickets[s].append(srv.submit_key(db_ids[s], key, outs[s][q]))
    return outs, tickets


def _collect(servers, tickets, timeout_ms):
    for srv, ts in zip(servers, tickets):
        for t in ts:
            rc = srv.wait(t, timeout_ms)
            if rc != PIR_OK:
                raise RuntimeError(f"request failed with status {rc}")


def run(n_records=1 << 20, record_bytes=32, n_queries=64, update_count=4096, seed=1, device=0,
        timeout_ms=120000):
    """Run the two-server exchange; returns a summary dict (checks included)."""
    rng = np.random.default_rng(seed)
    records = rng.integers(0, 256, (n_records, record_bytes), dtype=np.uint8)
    n_bits = dpf_domain_bits(n_records)
    ctxs = [Context(device), Context(device)]
    dbs, servers, db_ids = [], [], []
    try:
        for c in ctxs:
            db = c.load_db(records)
            srv = Server(c, q_max=64, max_wait_us=500, n_slots=2)
            dbs.append(db)
            servers.append(srv)
            db_ids.append(srv.add_db(db))

        # queries before the update; the update is pushed while they may still
        # be queued, then queries after it
        first = int(rng.integers(0, n_records - update_count + 1))
        new_records = rng.integers(0, 256, (update_count, record_bytes), dtype=np.uint8)
        idx_a = rng.integers(0, n_records, n_queries)
        idx_a[: min(8, n_queries)] = first + rng.integers(0, update_count, min(8, n_queries))
        idx_b = idx_a.copy()

        t0 = time.perf_counter()
        out_a, tick_a = _fetch(servers, db_ids, n_bits, idx_a, record_bytes)
        upd = [srv.update(i, first, new_records) for srv, i in zip(servers, db_ids)]
        out_b, tick_b = _fetch(servers, db_ids, n_bits, idx_b, record_bytes)
        _collect(servers, tick_a, timeout_ms)
        _collect(servers, [[u] for u in upd], timeout_ms)
        _collect(servers, tick_b, timeout_ms)
        wall = time.perf_counter() - t0

        after = records.copy()
        after[first:first + update_count] = new_records
        got_a = np.stack([reconstruct(out_a[0][q], out_a[1][q]) for q in range(n_queries)])
        got_b = np.stack([reconstruct(out_b[0][q], out_b[1][q]) for q in range(n_queries)])
        stats = [srv.stats() for srv in servers]
        replica_ok = all(np.array_equal(db.read(first, update_count), new_records) for db in dbs)
        return {
            "records": n_records, "record_bytes": record_bytes, "domain_bits": n_bits,
            "queries": 2 * n_queries, "wall_s": wall, "queries_per_s": 2 * n_queries / wall,
            "before_update_ok": bool(np.array_equal(got_a, records[idx_a])),
            "after_update_ok": bool(np.array_equal(got_b, after[idx_b])),
            "replicas_updated": bool(replica_ok),
            "key_bytes_per_query": int(2 * 64 * (n_bits + 1)),
            "server_stats": [{k: s[k] for k in ("completed", "batches", "key_requests", "updates_applied",
                                                  "p50_us", "p99_us", "h2d_bytes")} for s in stats],
        }
    finally:
        for srv in servers:
            srv.close()
        for db in dbs:
            db.free()
        for c in ctxs:
            c.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--records", type=int, default=1 << 20)
    ap.add_argument("--record-bytes", type=int, default=32)
    ap.add_argument("--queries", type=int, default=64)
    ap.add_argument("--update-count", type=int, default=4096)
    args = ap.parse_args()
    print(json.dumps(run(args.records, args.record_bytes, args.queries, args.update_count)), flush=True)


if __name__ == "__main__":
    main()
