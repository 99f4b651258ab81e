"""profile_summary.py's counter mode on a hand-made results database (host
logic only): the copy probe is the last copy dispatch, every tile shape of
a template counts as one kernel with --prefix, and --last averages over the
last dispatches only."""
import sqlite3

import profile_summary as PS


def _db(tmp_path, name, counter, rows):
    path = tmp_path / name
    con = sqlite3.connect(path)
    con.execute("create table kernels (dispatch_id integer, name text, start integer, duration integer)")
    con.execute("create table pmc_events (dispatch_id integer, counter_name text, counter_value real)")
    for did, kname, val in rows:
        con.execute("insert into kernels values (?, ?, ?, ?)", (did, kname, did * 10, 5))
        # two instances of the counter per dispatch, summed by the reader
        con.execute("insert into pmc_events values (?, ?, ?)", (did, counter, val / 2))
        con.execute("insert into pmc_events values (?, ?, ?)", (did, counter, val / 2))
    con.commit()
    con.close()
    return str(path)


ROWS = [
    (1, "__amd_rocclr_copyBuffer(a)", 1000.0),                 # an earlier, larger copy
    (2, "void eahp::k_gemm_nn_mfma<float, 2, 2, 4, 2>(x)", 10.0),
    (3, "void eahp::k_gemm_nn_mfma<float, 4, 1, 1, 1>(x)", 20.0),
    (4, "void eahp::k_gemm_nn_mfma<float, 2, 2, 4, 2>(x)", 30.0),
    (5, "void eahp::k_gemm_nn_mfma<float, 2, 2, 2, 2>(x)", 50.0),
    (6, "__amd_rocclr_copyBuffer(a)", 256.0),                  # the probe: last copy
]


def test_last_copy_is_the_probe(tmp_path):
    db = _db(tmp_path, "f.db", "FETCH_SIZE", ROWS)
    name, val = PS.last_dispatch(db, "FETCH_SIZE", "copy")
    assert name == "__amd_rocclr_copyBuffer"
    assert val == 256.0 * 1024.0


def test_prefix_groups_shapes_and_last_windows(tmp_path):
    db = _db(tmp_path, "f.db", "FETCH_SIZE", ROWS)
    group = "void eahp::k_gemm_nn_mfma<float"
    allv = PS.pmc(db, "FETCH_SIZE", group, 0)[group]
    assert allv == [10.0, 20.0, 30.0, 50.0]            # dispatch order, instances summed
    assert PS.pmc(db, "FETCH_SIZE", group, 2)[group] == [30.0, 50.0]
    # without a group every shape is its own kernel
    per = PS.pmc(db, "FETCH_SIZE")
    assert per["void eahp::k_gemm_nn_mfma<float, 2, 2, 4, 2>"] == [10.0, 30.0]
