"""Host logic of the profile summariser: the burst view of a kernel trace
keeps only launches that come in runs of back-to-back dispatches of one
kernel (a synthetic trace table stands in for rocprofv3's output)."""
import sqlite3

from paper_2110_06322_amd import profile_summary


def _trace(path, names_durations):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, duration integer)")
    t = 0
    for name, dur in names_durations:
        con.execute("insert into kernels values (?, ?, ?)", (name, t, dur))
        t += dur + 10
    con.commit()
    con.close()


def test_bursts_average_only_long_runs(tmp_path, capsys):
    db = str(tmp_path / "t.db")
    seq = [("k_apply_pipe<3,3>", 30000)] * 3 + [("k_other", 5000)]      # a short run
    seq += [("k_apply_pipe<3,3>", 12000)] * 60 + [("k_other", 5000)]    # a burst
    seq += [("k_apply_pipe<3,3>", 14000)] * 60                          # a burst at the end
    _trace(db, seq)
    profile_summary.bursts(db, "k_apply_pipe", 50)
    out = capsys.readouterr().out
    assert "runs=2 launches=120 of 123" in out
    assert "avg_us=13.000" in out


def test_bursts_reports_when_no_run_is_long_enough(tmp_path, capsys):
    db = str(tmp_path / "t.db")
    _trace(db, [("k_apply_pipe<3,3>", 1000), ("k_other", 1000)] * 5)
    profile_summary.bursts(db, "k_apply_pipe", 50)
    assert "no runs of 50 or more" in capsys.readouterr().out
