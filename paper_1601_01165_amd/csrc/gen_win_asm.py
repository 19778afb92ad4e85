#!/usr/bin/env python3
"""Generate the gfx950 inner step of the register-window dedispersion kernel.

The paper instantiates its kernel source from tuning parameters at run time
(Section 2.2).  Here the instantiation happens ahead of time: this script
writes ``win_asm.inc``, one inline-assembly step per (TP, DPW, NWIN,
weighted) variant, which ``engine.hip`` includes.

One step processes one input row (a channel in the forward map) for the
DPW output rows (DM trials) of one wave:

  1. load the lane's window of consecutive input samples from LDS into fixed
     VGPRs with 16-byte reads (only as many reads as the row's delay span
     needs, ``nl``);
  2. once they have landed, issue the scalar load of the next row's table
     entry (and weight), whose latency then hides behind the adds;
  3. turn VGPR index mode on and, for each of the DPW rows j, set the index
     to the row's window offset o_j (one SGPR each) and add the TP window
     registers starting at o_j into the row's TP accumulators:
        acc[j][i] += win[o_j + i]        (or fma(win[o_j + i], w, acc[j][i]))
     so each accumulator receives exactly one term per input row, in input
     row order, with one rounding per term.

A lane owns TP consecutive samples, so neighbouring lanes' windows start
4*TP bytes apart; TP/4 odd keeps the 16-byte LDS reads free of bank
conflicts.  Accumulators live in VGPRs v[ACC0 ...] and the window right
after them; the C++ side binds the accumulators with physical-register
constraints.  Table entry layout (ints): {window start, nl, o_0, ..., o_{DPW-1}}.
"""
import os
import sys

ACC0 = 32

# (TP samples per lane, DPW rows per wave, NWIN window registers)
VARIANTS = [
    (8, 8, 64),
    (16, 8, 72),
    (16, 4, 64),
    (8, 4, 48),
    (12, 4, 36),
    (12, 4, 48),
    (12, 8, 56),
    (20, 4, 44),
]


def entry_ints(dpw):
    n = dpw + 2
    return 4 if n <= 4 else 8 if n <= 8 else 16


def step(tp, dpw, nwin, weighted):
    """Return the C++ specialisation of win_step for one variant."""
    nacc = tp * dpw
    assert nacc % 16 == 0 and nwin % 4 == 0 and tp % 4 == 0
    w0 = ACC0 + nacc
    assert w0 + nwin <= 256
    nmin = tp // 4 + 1
    nmax = nwin // 4
    ent = entry_ints(dpw)
    lines = []
    # index mode keeps its index in M0, a register the compiler reserves for
    # itself (LDS DMA uses it): save it here and restore it at the end
    lines.append("s_mov_b32 %[m0s], m0")
    # window loads: the first nmin always, the rest while k < nl
    for k in range(nmin):
        lines.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[addr] offset:{16 * k}")
    for k in range(nmin, nmax):
        lines.append(f"s_cmp_le_u32 %[nl], {k}")
        lines.append("s_cbranch_scc1 .Lwin_loaded_%=")
        lines.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[addr] offset:{16 * k}")
    lines.append(".Lwin_loaded_%=:")
    lines.append("s_waitcnt lgkmcnt(0)")
    # the next row's table entry (and weight) load while the adds run; the
    # final wait leaves them complete when the step returns
    lines.append(f"s_load_dwordx{ent} %[nxt], %[nptr], 0x0")
    if weighted:
        lines.append("s_load_dword %[wn], %[wptr], 0x0")
    for j in range(dpw):
        if j == 0:
            lines.append("s_set_gpr_idx_on %[o0], gpr_idx(SRC0)")
        else:
            lines.append(f"s_set_gpr_idx_idx %[o{j}]")
        for i in range(tp):
            a = ACC0 + j * tp + i
            if weighted:
                lines.append(f"v_fma_f32 v{a}, v{w0 + i}, %[w], v{a}")
            else:
                lines.append(f"v_add_f32 v{a}, v{w0 + i}, v{a}")
    lines.append("s_set_gpr_idx_off")
    lines.append("s_mov_b32 m0, %[m0s]")
    lines.append("s_waitcnt lgkmcnt(0)")
    asm = "".join(f'    "{ln}\\n\\t"\n' for ln in lines)
    outs = ['[m0s] "=&s"(m0s)', '[nxt] "=&s"(nxt)']
    if weighted:
        outs.append('[wn] "=&s"(wn)')
    for q in range(nacc // 16):
        lo = ACC0 + 16 * q
        outs.append(f'[a{q}] "+{{v[{lo}:{lo + 15}]}}"(acc[{q}])')
    ins = ['[addr] "v"(addr)', '[nl] "s"(cur[1])', '[nptr] "s"(nptr)']
    for j in range(dpw):
        ins.append(f'[o{j}] "s"(cur[{2 + j}])')
    if weighted:
        ins.append('[w] "s"(w)')
        ins.append('[wptr] "s"(wptr)')
    clob = [f'"v{w0 + r}"' for r in range(nwin)] + ['"scc"']
    wflag = "true" if weighted else "false"
    etype = f"ent{ent}_t"
    return (
        f"template <>\n"
        f"__device__ __forceinline__ void win_step<{tp}, {dpw}, {nwin}, {wflag}>(v16f* acc, uint32_t addr,\n"
        f"    const {etype}& cur, const int32_t* nptr, {etype}& nxt, float w, const float* wptr, float& wn) {{\n"
        f"  uint32_t m0s;\n"
        f"  (void)w;\n"
        f"  (void)wptr;\n"
        f"  (void)wn;\n"
        f"  asm volatile(\n{asm}"
        f"    : {', '.join(outs)}\n"
        f"    : {', '.join(ins)}\n"
        f"    : {', '.join(clob)});\n"
        f"}}\n"
    )


# Pipelined variants (TP, DPW, NWIN window registers per bank): two register
# windows, the next input row's loads in flight while the current row is summed.
PIPE_VARIANTS = [
    (20, 4, 44),
    (12, 4, 36),
    (12, 8, 56),
]


def chunks(n):
    """Split n registers (a multiple of 4) into tuples of 16/8/4."""
    out = []
    for c in (16, 8, 4):
        while n >= c:
            out.append(c)
            n -= c
    return out


def bank_struct(nwin):
    fields = "".join(f"  v{c}f c{i};\n" for i, c in enumerate(chunks(nwin)))
    return f"template <> struct BankT<{nwin}> {{\n{fields}}};\n"


def bank_operands(name, base, nwin):
    ops, r = [], base
    for i, c in enumerate(chunks(nwin)):
        ops.append(f'[{name}{i}] "+{{v[{r}:{r + c - 1}]}}"({name}.c{i})')
        r += c
    return ops


def window_loads(w0, tp, nwin, label):
    """nmin unconditional 16-byte reads, then one more while k < nl."""
    lines = []
    nmin, nmax = tp // 4 + 1, nwin // 4
    for k in range(nmin):
        lines.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[addr] offset:{16 * k}")
    for k in range(nmin, nmax):
        lines.append(f"s_cmp_le_u32 %[nl], {k}")
        lines.append(f"s_cbranch_scc1 {label}")
        lines.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[addr] offset:{16 * k}")
    return lines


def asm_body(lines):
    return "".join(f'    "{ln}\\n\\t"\n' for ln in lines)


def pipe_step(tp, dpw, nwin, weighted):
    """Specialisation of win_pstep: load the next row's window into bank xb,
    fetch the entry two rows ahead, and sum the current row, whose offsets
    already include its bank (0 or nwin) and so select it through the index."""
    nacc = tp * dpw
    assert nacc % 16 == 0 and nwin % 4 == 0 and tp % 4 == 0
    wa = ACC0 + nacc
    wb = wa + nwin
    assert wb + nwin <= 256
    ent = entry_ints(dpw)
    lines = ["s_mov_b32 %[m0s], m0", "s_cmp_eq_u32 %[xb], 0", "s_cbranch_scc1 .Lpload_a_%="]
    lines += window_loads(wb, tp, nwin, ".Lpload_done_%=")
    lines += ["s_branch .Lpload_done_%=", ".Lpload_a_%=:"]
    lines += window_loads(wa, tp, nwin, ".Lpload_done_%=")
    lines.append(".Lpload_done_%=:")
    lines.append(f"s_load_dwordx{ent} %[nxt], %[nptr], 0x0")
    if weighted:
        lines.append("s_load_dword %[wn], %[wptr], 0x0")
    for j in range(dpw):
        lines.append("s_set_gpr_idx_on %[o0], gpr_idx(SRC0)" if j == 0 else f"s_set_gpr_idx_idx %[o{j}]")
        for i in range(tp):
            a = ACC0 + j * tp + i
            if weighted:
                lines.append(f"v_fma_f32 v{a}, v{wa + i}, %[w], v{a}")
            else:
                lines.append(f"v_add_f32 v{a}, v{wa + i}, v{a}")
    lines.append("s_set_gpr_idx_off")
    lines.append("s_mov_b32 m0, %[m0s]")
    lines.append("s_waitcnt lgkmcnt(0)")
    outs = ['[m0s] "=&s"(m0s)', '[nxt] "=&s"(nxt)']
    if weighted:
        outs.append('[wn] "=&s"(wn)')
    for q in range(nacc // 16):
        lo = ACC0 + 16 * q
        outs.append(f'[a{q}] "+{{v[{lo}:{lo + 15}]}}"(acc[{q}])')
    outs += bank_operands("ba", wa, nwin) + bank_operands("bb", wb, nwin)
    ins = ['[addr] "v"(addr)', '[nl] "s"(nl)', '[xb] "s"(xb)', '[nptr] "s"(nptr)']
    for j in range(dpw):
        ins.append(f'[o{j}] "s"(cur[{2 + j}])')
    if weighted:
        ins.append('[w] "s"(w)')
        ins.append('[wptr] "s"(wptr)')
    wflag = "true" if weighted else "false"
    etype = f"ent{ent}_t"
    return (
        f"template <>\n"
        f"__device__ __forceinline__ void win_pstep<{tp}, {dpw}, {nwin}, {wflag}>(v16f* acc, BankT<{nwin}>& ba,\n"
        f"    BankT<{nwin}>& bb, uint32_t addr, int nl, int xb, const {etype}& cur, const int32_t* nptr,\n"
        f"    {etype}& nxt, float w, const float* wptr, float& wn) {{\n"
        f"  uint32_t m0s;\n"
        f"  (void)w;\n"
        f"  (void)wptr;\n"
        f"  (void)wn;\n"
        f"  asm volatile(\n{asm_body(lines)}"
        f"    : {', '.join(outs)}\n"
        f"    : {', '.join(ins)}\n"
        f"    : \"scc\");\n"
        f"}}\n"
    )


def pipe_load(tp, dpw, nwin):
    """Specialisation of win_pload: the first row's window into bank 0."""
    wa = ACC0 + tp * dpw
    wb = wa + nwin
    lines = window_loads(wa, tp, nwin, ".Lpload_%=") + [".Lpload_%=:", "s_waitcnt lgkmcnt(0)"]
    outs = bank_operands("ba", wa, nwin) + bank_operands("bb", wb, nwin)
    return (
        f"template <>\n"
        f"__device__ __forceinline__ void win_pload<{tp}, {dpw}, {nwin}>(BankT<{nwin}>& ba, BankT<{nwin}>& bb,\n"
        f"    uint32_t addr, int nl) {{\n"
        f"  asm volatile(\n{asm_body(lines)}"
        f"    : {', '.join(outs)}\n"
        f"    : [addr] \"v\"(addr), [nl] \"s\"(nl)\n"
        f"    : \"scc\");\n"
        f"}}\n"
    )


def main(out_path):
    parts = [
        "// Generated by gen_win_asm.py: inner step of the register-window kernel.\n",
        "// Do not edit by hand.\n",
        "#pragma once\n\n",
        f"#define WIN_ACC0 {ACC0}\n\n",
        "// Table entry of one (wave tile, input row): {window start, loads, offset per row...}.\n",
        "typedef int32_t ent4_t __attribute__((ext_vector_type(4)));\n",
        "typedef int32_t ent8_t __attribute__((ext_vector_type(8)));\n",
        "typedef int32_t ent16_t __attribute__((ext_vector_type(16)));\n",
        "template <int DPW> struct EntT {\n",
        "  typedef typename std::conditional<(DPW + 2 <= 4), ent4_t,\n",
        "      typename std::conditional<(DPW + 2 <= 8), ent8_t, ent16_t>::type>::type type;\n",
        "  static constexpr int ints = DPW + 2 <= 4 ? 4 : DPW + 2 <= 8 ? 8 : 16;\n",
        "};\n\n",
        "// Loads the next row's entry from nptr into nxt (and its weight from wptr into wn)\n",
        "// while processing the current row described by cur.\n",
        "template <int TP, int DPW, int NWIN, bool WEIGHTED>\n",
        "__device__ __forceinline__ void win_step(v16f* acc, uint32_t addr, const typename EntT<DPW>::type& cur,\n",
        "    const int32_t* nptr, typename EntT<DPW>::type& nxt, float w, const float* wptr, float& wn);\n\n",
    ]
    for tp, dpw, nwin in VARIANTS:
        for weighted in (False, True):
            parts.append(step(tp, dpw, nwin, weighted))
            parts.append("\n")
    parts += [
        "typedef float v4f __attribute__((ext_vector_type(4)));\n",
        "typedef float v8f __attribute__((ext_vector_type(8)));\n",
        "typedef float v32f __attribute__((ext_vector_type(32)));\n",
        "// One register window: NWIN VGPRs at a fixed place, as a few register tuples.\n",
        "template <int NWIN> struct BankT;\n",
    ]
    for nwin in sorted({v[2] for v in PIPE_VARIANTS}):
        parts.append(bank_struct(nwin))
    parts += [
        "\n// Pipelined step: loads the window of the next row (LDS address addr, nl\n",
        "// 16-byte reads) into bank xb (0 or 1) while summing the current row (entry\n",
        "// cur, whose offsets include its bank's base, and weight w), and fetches the\n",
        "// entry (and weight) two rows ahead from nptr (wptr) into nxt (wn).\n",
        "// Everything has landed on return.\n",
        "template <int TP, int DPW, int NWIN, bool WEIGHTED>\n",
        "__device__ __forceinline__ void win_pstep(v16f* acc, BankT<NWIN>& ba, BankT<NWIN>& bb, uint32_t addr, int nl,\n",
        "    int xb, const typename EntT<DPW>::type& cur, const int32_t* nptr, typename EntT<DPW>::type& nxt,\n",
        "    float w, const float* wptr, float& wn);\n",
        "// Loads the first row's window into bank 0 and waits for it.\n",
        "template <int TP, int DPW, int NWIN>\n",
        "__device__ __forceinline__ void win_pload(BankT<NWIN>& ba, BankT<NWIN>& bb, uint32_t addr, int nl);\n\n",
    ]
    for tp, dpw, nwin in PIPE_VARIANTS:
        parts.append(pipe_load(tp, dpw, nwin))
        parts.append("\n")
        for weighted in (False, True):
            parts.append(pipe_step(tp, dpw, nwin, weighted))
            parts.append("\n")
    text = "".join(parts)
    if os.path.exists(out_path) and open(out_path).read() == text:
        return
    with open(out_path, "w") as f:
        f.write(text)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "win_asm.inc"))
