"""The profile summaries' source hash ignores comments and layout but not code."""
from paper_2009_07226_amd import pmc_summary as p


def test_code_only_drops_comments_keeps_literals():
    a = 'int a = 1; // note\n/* block\n comment */ const char *s = "// not a comment";\nchar c = \'/\';'
    b = 'int a = 1;\n  const char *s = "// not a comment"; char c = \'/\'; // other note'
    assert p.code_only(a) == p.code_only(b)
    assert "not a comment" in p.code_only(a)
    assert p.code_only("x = 1;") != p.code_only("x = 2;")


def test_kernel_sources_sha_is_stable():
    assert p.kernel_sources_sha() == p.kernel_sources_sha()
    assert len(p.kernel_sources_sha()) == 64


def test_sq_table_takes_the_first_a_and_at_launch(tmp_path):
    """Derived columns of the SQ table from a counter CSV in rocprofv3's
    layout: per-LDS-instruction cycles and per-group counts."""
    import json
    head = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size","Kernel_Id",'
            '"Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count","Accum_VGPR_Count",'
            '"SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"')
    vals = {5: (800.0, 100.0, 420.0, 20.0), 6: (1600.0, 200.0, 800.0, 10.0), 9: (1.0, 1.0, 1.0, 1.0)}
    rows = [head]
    for d, v in vals.items():
        for c, x in zip(p.SQ_COUNTERS, v):
            rows.append(f'{d},{d},"Agent 1",1,1,1,1024,3,"void xct::k_spmm<0, 16, 1, false, false>(xct::SpmmArgs)",'
                        f'1024,0,0,120,0,70,"{c}",{x},0,1')
    rows.append('1,1,"Agent 1",1,1,1,512,8,"__amd_rocclr_copyBuffer",512,0,0,8,0,32,"SQ_INSTS_LDS",7.0,0,1')
    csv_path = tmp_path / "sq.csv"
    csv_path.write_text("\n".join(rows) + "\n")
    bench = tmp_path / "bench.out"
    bench.write_text("[bench] text\n" + json.dumps({"padded_A": 2560, "padded_AT": 5120}) + "\n")
    out = tmp_path / "sq.md"
    p.sq_table([("f32", str(csv_path), str(bench))], str(out), "cmd", "w")
    lines = [ln for ln in out.read_text().splitlines() if ln.startswith("| f32")]
    assert len(lines) == 2
    a = [c.strip() for c in lines[0].split("|")[1:-1]]
    t = [c.strip() for c in lines[1].split("|")[1:-1]]
    # A: 10 groups; LDS cycles 420 / 100 instr; conflicts 20 / 100; VALU 800 / 10; LDS 100 / 10
    assert a[1] == "A" and a[-4:] == ["4.20", "0.200", "80.0", "10.0"]
    assert t[1] == "A^T" and t[-4:] == ["4.00", "0.050", "80.0", "10.0"]


def test_states_table_combines_two_passes(tmp_path):
    """Wavefront-state shares from two counter passes of the same launches:
    the three states divide SQ_WAVE_CYCLES, the instruction kinds divide
    SQ_ACTIVE_INST_ANY; the first k_spmm dispatch is A, the second A^T."""
    head = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size","Kernel_Id",'
            '"Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count","Accum_VGPR_Count",'
            '"SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"')

    def write(path, dispatches):
        rows = [head]
        for d, counters in dispatches.items():
            for c, x in counters.items():
                rows.append(f'{d},{d},"Agent 1",1,1,1,1024,3,"void xct::k_spmm<0, 16, 1, false, false>(xct::SpmmArgs)",'
                            f'1024,0,0,120,0,70,"{c}",{x},0,1')
        path.write_text("\n".join(rows) + "\n")

    a = {"SQ_WAVE_CYCLES": 1000.0, "SQ_WAIT_ANY": 500.0, "SQ_WAIT_INST_ANY": 250.0, "SQ_ACTIVE_INST_ANY": 250.0,
         "SQ_ACTIVE_INST_VALU": 125.0, "SQ_ACTIVE_INST_LDS": 25.0}
    at = {"SQ_WAVE_CYCLES": 2000.0, "SQ_WAIT_ANY": 400.0, "SQ_WAIT_INST_ANY": 600.0, "SQ_ACTIVE_INST_ANY": 1000.0,
          "SQ_ACTIVE_INST_VALU": 700.0, "SQ_ACTIVE_INST_LDS": 100.0}
    write(tmp_path / "a.csv", {11: dict(a, SQ_ACTIVE_INST_VMEM=10.0), 12: dict(at, SQ_ACTIVE_INST_VMEM=20.0)})
    write(tmp_path / "b.csv", {21: {"SQ_ACTIVE_INST_SCA": 50.0, "SQ_WAIT_INST_LDS": 30.0},
                               22: {"SQ_ACTIVE_INST_SCA": 100.0, "SQ_WAIT_INST_LDS": 200.0}})
    out = tmp_path / "s.md"
    p.states_table([("f32", str(tmp_path / "a.csv"), str(tmp_path / "b.csv"))], str(out), "cmd", "w")
    lines = [[c.strip() for c in ln.split("|")[1:-1]] for ln in out.read_text().splitlines() if ln.startswith("| f32")]
    assert lines[0][1:] == ["A", "50.0%", "25.0%", "25.0%", "50.0%", "10.0%", "4.0%", "20.0%", "3.0%"]
    assert lines[1][1:] == ["A^T", "20.0%", "30.0%", "50.0%", "70.0%", "10.0%", "2.0%", "10.0%", "10.0%"]
