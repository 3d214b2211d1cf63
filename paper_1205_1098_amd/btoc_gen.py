"""Code generation for compiled BTO programs: every fused matrix pass of a
program becomes an emitted HIP loop nest.

``btoc.compile_spec(text, target="generated")`` schedules a program for
emitted passes: the products of one matrix at one point of the schedule all
share its sweep (any number of row dots and column sums), and an update of
any rank is either stored by the sweep that forms it or contracted, i.e.
formed in registers by every sweep that reads it and never written
(Section III-E).  ``emit`` writes the HIP source of those passes (the loop
nest of Section III-C, with the statement bodies written out term by term),
``build`` compiles it with hipcc into a shared library with the C interface
of include/btog.h, and ``run`` executes the program: the matrix passes in
the generated library, the vector statements through libbto's vector
kernels.

The partition of each generated loop nest (the tile shape of a workgroup
and the band height: the partitioned loop and its thread count, Section
III-C) is a run-time choice: the library is compiled for every tile shape in
``SHAPES``, and a genome, one (shape, band height) per pass, selects them.
``tune`` searches genomes with the MFGA of Section IV (tune.mfga_genes);
every candidate's outputs are checked against the default genome's.

Libraries are built ahead of use (``build_all`` for the programs in
``bto_specs.GENERATED``, called by the package build) into
``paper_1205_1098_amd/gen``, named by program and source digest.
"""

from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess

from .btoc import ONE, Pass, Program, SpecError, compile_spec

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
GEN_DIR = os.path.join(PKG, "gen")
SRC_DIR = os.path.join(ROOT, "_build", "gen")
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         f"-I{INCLUDE}", f"-I{CSRC}"]

#: the tile shapes every generated pass is compiled for: (kv, depth, waves
#: across, waves down); a block is 128 * kv * waves_across columns
SHAPES = [(1, 2, 1, 16), (2, 2, 1, 8), (2, 4, 1, 4), (2, 2, 4, 4), (4, 4, 4, 1),
          (4, 2, 4, 2), (4, 2, 4, 4), (1, 4, 4, 1), (2, 2, 2, 8), (4, 2, 2, 4), (4, 2, 2, 8)]
#: band heights the search tries
RB_CHOICES = (4, 8, 16, 32, 64, 128, 256, 512)
MAX_TERMS, MAX_RED = 8, 8
ABI_VERSION = 1


# ---- the passes as the generator sees them ------------------------------------------

def gen_passes(prog: Program) -> list:
    """The program's matrix passes, in program order."""
    if prog.target != "generated":
        raise SpecError("emit needs a program compiled with target='generated'")
    passes = [s for s in prog.steps if isinstance(s, Pass)]
    for k, p in enumerate(passes):
        if len(p.terms) > MAX_TERMS or len(p.rows) > MAX_RED or len(p.cols) > MAX_RED:
            raise SpecError(f"pass {k}: more terms or reductions than a generated pass takes")
    return passes


def layout(p: Pass) -> tuple:
    """(update terms formed by the pass, stored?, row dots, column sums)."""
    nterms = len(p.terms) if (p.store or p.contract) else 0
    return nterms, bool(p.store), len(p.rows), len(p.cols)


def _scalar_expr(coef, scalars: list) -> str:
    """C expression of a coefficient (a literal times scalar inputs)."""
    lit, names = coef
    parts = [repr(float(lit))]
    for s in names:
        parts.append(f"sc[{scalars.index(s)}]")
    return " * ".join(parts)


# ---- emission ------------------------------------------------------------------------

_PRELUDE = """\
#include <stdint.h>
#include <string>

#include "bto.h"
#include "btog.h"
#include "bto_dev.hpp"
#include "bto_tile.hpp"

using namespace bto;

namespace {

thread_local std::string t_err;

bto_status gfail(bto_status s, const char *msg)
{
    t_err = msg;
    return s;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t r256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int kGenShapeCount = %(nshapes)d;
constexpr int kGenShapes[kGenShapeCount][4] = {%(shapes)s};

// One finish job: out[i] = scale * sum_k P[k * len + i] (+ add_scale * add[i]),
// the parts added in a fixed order (four interleaved runs of k, then the
// four run sums in order), 64 outputs per workgroup.
struct Job {
    const double *P;
    int64_t nparts, len;
    double scale, add_scale;
    const double *add;
    double *out;
};
constexpr int kMaxJobs = 2 * BTOG_MAX_RED;
struct Jobs {
    Job j[kMaxJobs];
    int64_t first[kMaxJobs + 1];   // first workgroup of each job
    int count;
};

__global__ __launch_bounds__(256) void gen_finish(Jobs f)
{
    __shared__ double lds[4][64];
    int k = 0;
    while (k + 1 < f.count && (int64_t)blockIdx.x >= f.first[k + 1])
        ++k;
    const Job &j = f.j[k];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t idx = ((int64_t)blockIdx.x - f.first[k]) * 64 + lane;
    const int64_t q = (j.nparts + 3) / 4;
    const int64_t k0 = wave * q;
    const int64_t k1 = k0 + q < j.nparts ? k0 + q : j.nparts;
    double s = 0.0;
    if (idx < j.len) {
        const double *p = j.P + idx;
        for (int64_t t = k0; t < k1; ++t)
            s += p[t * j.len];
    }
    lds[wave][lane] = s;
    lds_barrier();
    if (wave == 0 && idx < j.len) {
        const double t = ((lds[0][lane] + lds[1][lane]) + lds[2][lane]) + lds[3][lane];
        j.out[idx] = j.add ? j.scale * t + j.add_scale * j.add[idx] : j.scale * t;
    }
}

void launch_jobs(Jobs &f, hipStream_t st)
{
    int64_t blocks = 0;
    for (int k = 0; k < f.count; ++k) {
        f.first[k] = blocks;
        blocks += cdiv(f.j[k].len, 64);
    }
    f.first[f.count] = blocks;
    if (blocks > 0)
        gen_finish<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(f);
}

bool shape_ok(int shape, int rb, bool rowdots)
{
    if (shape < 0 || shape >= kGenShapeCount)
        return false;
    const int wr = kGenShapes[shape][3];
    if (rb < wr || rb %% wr != 0 || rb > 4096)
        return false;
    return !(rowdots && rb / wr > kWave);
}

int64_t wave_cols(int shape) { return 128 * (int64_t)kGenShapes[shape][0]; }

}  // namespace
"""


def _emit_pass(k: int, p: Pass, scalars: list) -> str:
    """The loop nest of pass k: its argument block, the row loop of one
    wave, the workgroup tile, the launch and the finish jobs."""
    R, store, P, Q = layout(p)
    L = []
    w = L.append
    desc = []
    if R:
        desc.append(("B = " if store else "M = ") + p.base + " + " +
                    " + ".join(f"{u} {v}'" for u, v in p.terms) +
                    (" (stored)" if store else " (contracted)"))
    for r in p.rows:
        desc.append(f"{r['out']} = row dots with {r['x']}")
    for c in p.cols:
        desc.append(f"{c['out']} = column sums with {c['y']}")
    w(f"// ---- pass {k}: one sweep of {p.base}: " + "; ".join(desc))
    w("namespace {")
    w(f"struct P{k}Args {{")
    w("    int64_t m, n, lda, ldb;")
    w("    const double *A;")
    w("    double *B;")
    for r in range(R):
        w(f"    const double *u{r}, *v{r};")
    for q in range(P):
        w(f"    const double *x{q};")
        w(f"    double *prow{q};")
    for q in range(Q):
        w(f"    const double *y{q};")
        w(f"    double *pcol{q};")
    w("};")
    w("")
    # the rows of one wave
    w("template <int KV, int D, bool VEC, bool FULL>")
    w(f"__device__ __forceinline__ void p{k}_rows(const P{k}Args &a, int64_t c0, int64_t r0, "
      f"int64_t r1, int lane, d2 (&acc)[{max(Q, 1)}][KV], double (&mine)[{max(P, 1)}])")
    w("{")
    w("    const int64_t n = a.n;")
    for r in range(R):
        w(f"    d2 v{r}[KV];")
    for q in range(P):
        w(f"    d2 x{q}[KV];")
    w("#pragma unroll")
    w("    for (int k = 0; k < KV; ++k) {")
    w("        const int64_t j = c0 + 2 * (lane + kWave * k);")
    for r in range(R):
        w(f"        v{r}[k] = load_vec_pair(a.v{r}, j, n);")
    for q in range(P):
        w(f"        x{q}[k] = load_vec_pair(a.x{q}, j, n);")
    w("    }")
    w("    auto load_row = [&](int64_t i, d2 (&dst)[KV]) {")
    w("        const double *row = a.A + i * a.lda;")
    w("#pragma unroll")
    w("        for (int k = 0; k < KV; ++k)")
    w("            dst[k] = load_pair<VEC, FULL>(row, c0 + 2 * (lane + kWave * k), n);")
    w("    };")
    w("    d2 ring[D][KV];")
    w("#pragma unroll")
    w("    for (int q = 0; q < D; ++q) {")
    w("        if (r0 + q < r1) {")
    w("            load_row(r0 + q, ring[q]);")
    w("        } else {")
    w("#pragma unroll")
    w("            for (int k = 0; k < KV; ++k)")
    w("                ring[q][k] = d2{0.0, 0.0};")
    w("        }")
    w("    }")
    w("    for (int64_t i0 = r0; i0 < r1; i0 += D) {")
    w("#pragma unroll")
    w("        for (int q = 0; q < D; ++q) {")
    w("            const int64_t i = i0 + q;")
    w("            if (i >= r1)")
    w("                break;")
    w("            d2 b[KV];")
    w("#pragma unroll")
    w("            for (int k = 0; k < KV; ++k)")
    w("                b[k] = ring[q][k];")
    w("            if (i + D < r1)")
    w("                load_row(i + D, ring[q]);")
    if R:
        w("            // the update, its terms added left to right")
        for r in range(R):
            w(f"            const double su{r} = ld_uniform(a.u{r} + i);")
        w("#pragma unroll")
        w("            for (int k = 0; k < KV; ++k) {")
        for r in range(R):
            w(f"                b[k] = b[k] + su{r} * v{r}[k];")
        w("            }")
    if store:
        w("            double *brow = a.B + i * a.ldb;")
        w("#pragma unroll")
        w("            for (int k = 0; k < KV; ++k)")
        w("                store_pair<VEC, FULL>(brow, c0 + 2 * (lane + kWave * k), n, b[k]);")
    for q in range(Q):
        w(f"            const double sy{q} = ld_uniform(a.y{q} + i);")
        w("#pragma unroll")
        w("            for (int k = 0; k < KV; ++k)")
        w(f"                acc[{q}][k] += b[k] * sy{q};")
    if P == 1:
        w("            {")
        w("                double s = 0.0;")
        w("#pragma unroll")
        w("                for (int k = 0; k < KV; ++k) {")
        w("                    s += b[k].x * x0[k].x;")
        w("                    s += b[k].y * x0[k].y;")
        w("                }")
        w("                s = wave_sum(s);")
        w("                if (lane == (int)(i - r0))")
        w("                    mine[0] = s;")
        w("            }")
    elif P > 1:
        # the row's dots reduced across the wave together
        w("            {")
        w(f"                double s[{P}], t[{P}];")
        for q in range(P):
            w(f"                s[{q}] = 0.0;")
            w("#pragma unroll")
            w("                for (int k = 0; k < KV; ++k) {")
            w(f"                    s[{q}] += b[k].x * x{q}[k].x;")
            w(f"                    s[{q}] += b[k].y * x{q}[k].y;")
            w("                }")
        w(f"                wave_sums<{P}>(s, t);")
        w("                if (lane == (int)(i - r0)) {")
        for q in range(P):
            w(f"                    mine[{q}] = t[{q}];")
        w("                }")
        w("            }")
    w("        }")
    w("    }")
    w("}")
    w("")
    # the workgroup tile
    w("template <int KV, int D, int WC, int WR, bool VEC>")
    w(f"__global__ __launch_bounds__(kWave * WC * WR) void p{k}_kernel(P{k}Args a, int rb)")
    w("{")
    if Q:
        w("    constexpr int CTW = 128 * KV, CTB = WC * CTW, NT = kWave * WC * WR;")
        w("    __shared__ double lds[WR > 1 ? WR * CTB : 1];")
    else:
        w("    constexpr int CTW = 128 * KV;")
    w("    const int lane = threadIdx.x & 63;")
    w("    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);")
    w("    const int wc = wave % WC, wr = wave / WC;")
    w("    const int64_t band = blockIdx.y, cblk = blockIdx.x;")
    w("    const int64_t ctw = cblk * WC + wc;")
    w("    const int64_t c0 = ctw * CTW;")
    w("    const int rpw = rb / WR;")
    w("    const int64_t r0 = band * rb + (int64_t)wr * rpw;")
    w("    const int64_t r1 = r0 + rpw < a.m ? r0 + rpw : a.m;")
    w(f"    d2 acc[{max(Q, 1)}][KV];")
    w(f"    double mine[{max(P, 1)}];")
    w("#pragma unroll")
    w(f"    for (int q = 0; q < {max(Q, 1)}; ++q)")
    w("#pragma unroll")
    w("        for (int k = 0; k < KV; ++k)")
    w("            acc[q][k] = d2{0.0, 0.0};")
    w("#pragma unroll")
    w(f"    for (int q = 0; q < {max(P, 1)}; ++q)")
    w("        mine[q] = 0.0;")
    w("    if (c0 < a.n) {")
    w("        if (c0 + CTW <= a.n)")
    w(f"            p{k}_rows<KV, D, VEC, true>(a, c0, r0, r1, lane, acc, mine);")
    w("        else")
    w(f"            p{k}_rows<KV, D, VEC, false>(a, c0, r0, r1, lane, acc, mine);")
    w("    }")
    if P:
        w("    if (c0 < a.n && lane < r1 - r0) {")
        for q in range(P):
            w(f"        a.prow{q}[ctw * a.m + r0 + lane] = mine[{q}];")
        w("    }")
    for q in range(Q):
        w("    if constexpr (WR == 1) {")
        w("#pragma unroll")
        w("        for (int k = 0; k < KV; ++k) {")
        w("            const int64_t j = c0 + 2 * (lane + kWave * k);")
        w(f"            if (j < a.n) a.pcol{q}[band * a.n + j] = acc[{q}][k].x;")
        w(f"            if (j + 1 < a.n) a.pcol{q}[band * a.n + j + 1] = acc[{q}][k].y;")
        w("        }")
        w("    } else {")
        w("        // the row groups' column sums meet in LDS, added in row-group order")
        w("#pragma unroll")
        w("        for (int k = 0; k < KV; ++k) {")
        w("            const int c = wc * CTW + 2 * (lane + kWave * k);")
        w(f"            lds[wr * CTB + c] = acc[{q}][k].x;")
        w(f"            lds[wr * CTB + c + 1] = acc[{q}][k].y;")
        w("        }")
        w("        lds_barrier();")
        w("        for (int c = threadIdx.x; c < CTB; c += NT) {")
        w("            const int64_t j = cblk * CTB + c;")
        w("            if (j < a.n) {")
        w("                double s = lds[c];")
        w("#pragma unroll")
        w("                for (int r = 1; r < WR; ++r)")
        w("                    s += lds[r * CTB + c];")
        w(f"                a.pcol{q}[band * a.n + j] = s;")
        w("            }")
        w("        }")
        w("        lds_barrier();")
        w("    }")
    w("}")
    w("")
    # launch for one shape
    w("template <int KV, int D, int WC, int WR>")
    w(f"void p{k}_launch(const P{k}Args &a, int rb, hipStream_t st)")
    w("{")
    w("    const dim3 grid((unsigned)cdiv(a.n, (int64_t)WC * 128 * KV), (unsigned)cdiv(a.m, rb));")
    w("    bool vec = ((uintptr_t)a.A & 15u) == 0 && (a.lda % 2 == 0 || a.m <= 1);")
    if store:
        w("    vec = vec && ((uintptr_t)a.B & 15u) == 0 && (a.ldb % 2 == 0 || a.m <= 1);")
    w("    if (vec)")
    w(f"        p{k}_kernel<KV, D, WC, WR, true><<<grid, dim3(kWave * WC * WR), 0, st>>>(a, rb);")
    w("    else")
    w(f"        p{k}_kernel<KV, D, WC, WR, false><<<grid, dim3(kWave * WC * WR), 0, st>>>(a, rb);")
    w("}")
    w("")
    w(f"void p{k}_dispatch(int shape, const P{k}Args &a, int rb, hipStream_t st)")
    w("{")
    w("    switch (shape) {")
    for s, (kv, d, wc, wr) in enumerate(SHAPES):
        w(f"    case {s}: p{k}_launch<{kv}, {d}, {wc}, {wr}>(a, rb, st); break;")
    w("    default: break;")
    w("    }")
    w("}")
    w("")
    # workspace and run
    w(f"size_t p{k}_ws(int64_t m, int64_t n, int shape, int rb)")
    w("{")
    terms = []
    if P:
        w("    const int64_t ncols = n > 0 ? cdiv(n, wave_cols(shape)) : 0;")
        terms.append(f"{P} * r256((size_t)(ncols * m) * 8)")
    else:
        w("    (void)shape;")
    if Q:
        w("    const int64_t nbands = m > 0 ? cdiv(m, rb) : 0;")
        terms.append(f"{Q} * r256((size_t)(nbands * n) * 8)")
    else:
        w("    (void)rb;")
    w(f"    return {' + '.join(terms) if terms else '0'};")
    w("}")
    w("")
    w(f"bto_status p{k}_run(const btog_pass_args *g, int shape, int rb, void *ws, "
      "size_t wsb, hipStream_t st)")
    w("{")
    w("    const int64_t m = g->m, n = g->n;")
    w("    if (m < 0 || n < 0)")
    w("        return gfail(BTO_ERR_INVALID_ARG, \"negative size\");")
    w("    if (g->lda < (n > 1 ? n : 1))")
    w("        return gfail(BTO_ERR_INVALID_ARG, \"lda below max(1, n)\");")
    w(f"    if (!shape_ok(shape, rb, {'true' if P else 'false'}))")
    w("        return gfail(BTO_ERR_INVALID_ARG, \"tile shape / band height not supported\");")
    nsc = len(scalars)
    if nsc > 0:
        w(f"    if (g->scalars == nullptr || g->nscalars < {nsc})")
        w("        return gfail(BTO_ERR_INVALID_ARG, \"too few scalars\");")
    w("    const bool some = m > 0 && n > 0;")
    w("    if (some && g->A == nullptr)")
    w("        return gfail(BTO_ERR_INVALID_ARG, \"A is NULL\");")
    if store:
        w("    if (g->ldb < (n > 1 ? n : 1))")
        w("        return gfail(BTO_ERR_INVALID_ARG, \"ldb below max(1, n)\");")
        w("    if (some && g->B == nullptr)")
        w("        return gfail(BTO_ERR_INVALID_ARG, \"B is NULL\");")
        w("    if (g->B == g->A && g->ldb != g->lda && m > 1)")
        w("        return gfail(BTO_ERR_ALIAS, \"B == A requires ldb == lda\");")
    for r in range(R):
        w(f"    if ((m > 0 && g->u[{r}] == nullptr) || (n > 0 && g->v[{r}] == nullptr))")
        w(f"        return gfail(BTO_ERR_INVALID_ARG, \"update term {r} is NULL\");")
    for q in range(P):
        w(f"    if ((n > 0 && g->x[{q}] == nullptr) || (m > 0 && g->row_out[{q}] == nullptr))")
        w(f"        return gfail(BTO_ERR_INVALID_ARG, \"row dot {q}: NULL operand\");")
    for q in range(Q):
        w(f"    if ((m > 0 && g->y[{q}] == nullptr) || (n > 0 && g->col_out[{q}] == nullptr))")
        w(f"        return gfail(BTO_ERR_INVALID_ARG, \"column sum {q}: NULL operand\");")
    w("    const int64_t nbands = m > 0 ? cdiv(m, rb) : 0;")
    w("    if (nbands > 65535)")
    w("        return gfail(BTO_ERR_UNSUPPORTED, \"more row bands than a launch grid holds\");")
    w(f"    const size_t need = p{k}_ws(m, n, shape, rb);")
    w("    if (wsb < need)")
    w("        return gfail(BTO_ERR_WORKSPACE, \"workspace too small\");")
    w("    if (need > 0 && (ws == nullptr || ((uintptr_t)ws & 255u)))")
    w("        return gfail(BTO_ERR_INVALID_ARG, \"workspace NULL or not 256-byte aligned\");")
    if nsc:
        w("    const double *sc = g->scalars;")
    w(f"    P{k}Args a{{}};")
    w("    a.m = m;")
    w("    a.n = n;")
    w("    a.lda = g->lda;")
    w("    a.ldb = g->ldb;")
    w("    a.A = g->A;")
    w(f"    a.B = {'g->B' if store else 'nullptr'};")
    for r in range(R):
        w(f"    a.u{r} = g->u[{r}];")
        w(f"    a.v{r} = g->v[{r}];")
    w("    char *base = static_cast<char *>(ws);")
    if P:
        w("    const int64_t ncols = n > 0 ? cdiv(n, wave_cols(shape)) : 0;")
    for q in range(P):
        w(f"    a.x{q} = g->x[{q}];")
        w(f"    a.prow{q} = reinterpret_cast<double *>(base);")
        w("    base += r256((size_t)(ncols * m) * 8);")
    for q in range(Q):
        w(f"    a.y{q} = g->y[{q}];")
        w(f"    a.pcol{q} = reinterpret_cast<double *>(base);")
        w("    base += r256((size_t)(nbands * n) * 8);")
    w("    if (some)")
    w(f"        p{k}_dispatch(shape, a, rb, st);")
    w("    Jobs f{};")
    w("    f.count = 0;")
    for q, r in enumerate(p.rows):
        addsc = _scalar_expr(r["add_scale"], scalars) if r.get("add") is not None else "0.0"
        w(f"    f.j[f.count++] = Job{{a.prow{q}, ncols, m, {_scalar_expr(r['scale'], scalars)}, "
          f"{addsc}, g->row_add[{q}], g->row_out[{q}]}};")
    for q, c in enumerate(p.cols):
        addsc = _scalar_expr(c["add_scale"], scalars) if c.get("add") is not None else "0.0"
        w(f"    f.j[f.count++] = Job{{a.pcol{q}, nbands, n, {_scalar_expr(c['scale'], scalars)}, "
          f"{addsc}, g->col_add[{q}], g->col_out[{q}]}};")
    w("    launch_jobs(f, st);")
    w("    const hipError_t e = hipGetLastError();")
    w("    if (e != hipSuccess)")
    w("        return gfail(BTO_ERR_HIP, hipGetErrorString(e));")
    w("    return BTO_SUCCESS;")
    w("}")
    w("}  // namespace")
    return "\n".join(L)


def emit(prog: Program) -> str:
    """The HIP source of a program's passes (see include/btog.h)."""
    passes = gen_passes(prog)
    scalars = [n for n in prog.inputs if prog.kinds[n] == "scalar"]
    body = [_emit_pass(k, p, scalars) for k, p in enumerate(passes)]
    shapes = ", ".join("{%d, %d, %d, %d}" % s for s in SHAPES)
    head = (f"// Generated by btoc from the specification of {prog.name}: "
            f"{len(passes)} fused matrix pass(es).\n"
            "// Regenerate with python -m paper_1205_1098_amd.btoc_gen; do not edit.\n")
    layouts = ", ".join("{%d, %d, %d, %d}" % layout(p) for p in passes)
    digest = hashlib.sha256(("\n".join(body) + shapes).encode()).hexdigest()[:16]
    tail = [
        "namespace {",
        f"constexpr int kPasses = {len(passes)};",
        f"constexpr int kLayout[kPasses][4] = {{{layouts}}};",
        "}  // namespace",
        "",
        'extern "C" {',
        "",
        f"int btog_abi_version(void) {{ return {ABI_VERSION}; }}",
        f'const char *btog_program(void) {{ return "{prog.name}"; }}',
        f'const char *btog_source_digest(void) {{ return "{digest}"; }}',
        "int btog_pass_count(void) { return kPasses; }",
        "int btog_shape_count(void) { return kGenShapeCount; }",
        "const char *btog_last_error(void) { return t_err.c_str(); }",
        "",
        "bto_status btog_pass_layout(int pass, int counts[4])",
        "{",
        "    if (pass < 0 || pass >= kPasses || !counts)",
        '        return gfail(BTO_ERR_INVALID_ARG, "no such pass");',
        "    for (int i = 0; i < 4; ++i)",
        "        counts[i] = kLayout[pass][i];",
        "    return BTO_SUCCESS;",
        "}",
        "",
        "bto_status btog_shape(int shape, int *kv, int *depth, int *waves_across, int *waves_down)",
        "{",
        "    if (shape < 0 || shape >= kGenShapeCount)",
        '        return gfail(BTO_ERR_INVALID_ARG, "no such shape");',
        "    if (kv) *kv = kGenShapes[shape][0];",
        "    if (depth) *depth = kGenShapes[shape][1];",
        "    if (waves_across) *waves_across = kGenShapes[shape][2];",
        "    if (waves_down) *waves_down = kGenShapes[shape][3];",
        "    return BTO_SUCCESS;",
        "}",
        "",
        "int btog_config_ok(int pass, int shape, int rb)",
        "{",
        "    if (pass < 0 || pass >= kPasses)",
        "        return 0;",
        "    return shape_ok(shape, rb, kLayout[pass][2] > 0) ? 1 : 0;",
        "}",
        "",
        "size_t btog_pass_workspace_bytes(int pass, int64_t m, int64_t n, int shape, int rb)",
        "{",
        "    if (m < 0 || n < 0 || !btog_config_ok(pass, shape, rb))",
        "        return 0;",
        "    switch (pass) {",
    ]
    for k in range(len(passes)):
        tail.append(f"    case {k}: return p{k}_ws(m, n, shape, rb);")
    tail += [
        "    default: return 0;",
        "    }",
        "}",
        "",
        "bto_status btog_run_pass(int pass, const btog_pass_args *args, int shape, int rb, "
        "void *ws,",
        "                         size_t ws_bytes, hipStream_t stream)",
        "{",
        "    t_err.clear();",
        "    if (!args)",
        '        return gfail(BTO_ERR_INVALID_ARG, "args is NULL");',
        "    switch (pass) {",
    ]
    for k in range(len(passes)):
        tail.append(f"    case {k}: return p{k}_run(args, shape, rb, ws, ws_bytes, stream);")
    tail += [
        "    default:",
        '        return gfail(BTO_ERR_INVALID_ARG, "no such pass");',
        "    }",
        "}",
        "",
        '}  // extern "C"',
        "",
    ]
    return (head + (_PRELUDE % {"nshapes": len(SHAPES), "shapes": shapes}) + "\n"
            + "\n\n".join(body) + "\n\n" + "\n".join(tail))


# ---- building ------------------------------------------------------------------------

def digest(source: str) -> str:
    return hashlib.sha256(source.encode()).hexdigest()[:12]


def library_path(prog: Program, source: str | None = None) -> str:
    source = emit(prog) if source is None else source
    return os.path.join(GEN_DIR, f"libbtog_{prog.name.lower()}_{digest(source)}.so")


def build(prog: Program, verbose: bool = False, force: bool = False) -> str:
    """Emit and compile a program's library (once per source); its path."""
    source = emit(prog)
    path = library_path(prog, source)
    if os.path.exists(path) and not force:
        return path
    os.makedirs(GEN_DIR, exist_ok=True)
    os.makedirs(SRC_DIR, exist_ok=True)
    src = os.path.join(SRC_DIR, os.path.basename(path)[:-3] + ".hip")
    with open(src, "w") as f:
        f.write(source)
    tmp = path + ".tmp"
    cmd = [HIPCC, *FLAGS, src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(line for line in r.stderr.splitlines() if noise not in line)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    os.replace(tmp, path)
    return path


def build_all(verbose: bool = False, workers: int = 4, force: bool = True) -> list:
    """Build the libraries of the generated programs the package ships
    (bto_specs.GENERATED), and remove generated libraries of sources that
    are no longer current."""
    import concurrent.futures as cf

    from . import bto_specs

    progs = [compile_spec(t, target="generated") for t in bto_specs.GENERATED.values()]
    with cf.ThreadPoolExecutor(max_workers=max(1, min(workers, len(progs)))) as ex:
        paths = list(ex.map(lambda p: build(p, verbose, force), progs))
    keep = {os.path.basename(p) for p in paths}
    for f in os.listdir(GEN_DIR):
        if f.startswith("libbtog_") and f.endswith(".so") and f not in keep:
            os.remove(os.path.join(GEN_DIR, f))
    return paths


def main(argv=None) -> int:
    """python -m paper_1205_1098_amd.btoc_gen [SPEC] [--build]

    Prints the HIP source generated for a specification file (or one of
    bto_specs.GENERATED by name); --build compiles it (or, with no SPEC,
    every program of bto_specs.GENERATED)."""
    import argparse

    from . import bto_specs

    ap = argparse.ArgumentParser(description="HIP source of a BTO specification's passes")
    ap.add_argument("spec", nargs="?")
    ap.add_argument("--build", action="store_true")
    ap.add_argument("--tune", nargs="*", default=None, metavar="NAME",
                    help="search the genomes of these programs of bto_specs.GENERATED (all "
                         "when none is named) on the device at --n and write the tuned table")
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--table", default=TUNED_TABLE)
    args = ap.parse_args(argv)
    if args.tune is not None:
        return _tune_main(args.tune or sorted(bto_specs.GENERATED), args.n, args.table)
    if args.spec is None:
        if args.build:
            for p in build_all(verbose=True):
                print(p)
        return 0
    text = bto_specs.GENERATED.get(args.spec)
    if text is None:
        with open(args.spec) as f:
            text = f.read()
    prog = compile_spec(text, target="generated")
    if args.build:
        print(build(prog, verbose=True))
    else:
        print(emit(prog))
    return 0


# ---- loading and running ---------------------------------------------------------------

_i64, _int, _ptr, _sz, _dbl = (ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                               ctypes.c_double)


class PassArgs(ctypes.Structure):
    """btog_pass_args."""
    _fields_ = [("m", _i64), ("n", _i64), ("lda", _i64), ("ldb", _i64),
                ("A", _ptr), ("B", _ptr),
                ("u", _ptr * MAX_TERMS), ("v", _ptr * MAX_TERMS),
                ("x", _ptr * MAX_RED), ("row_out", _ptr * MAX_RED), ("row_add", _ptr * MAX_RED),
                ("y", _ptr * MAX_RED), ("col_out", _ptr * MAX_RED), ("col_add", _ptr * MAX_RED),
                ("scalars", ctypes.POINTER(_dbl)), ("nscalars", _int)]


_SIGS = {
    "btog_abi_version": ([], _int),
    "btog_program": ([], ctypes.c_char_p),
    "btog_source_digest": ([], ctypes.c_char_p),
    "btog_pass_count": ([], _int),
    "btog_pass_layout": ([_int, ctypes.POINTER(_int)], _int),
    "btog_shape_count": ([], _int),
    "btog_shape": ([_int] + [ctypes.POINTER(_int)] * 4, _int),
    "btog_config_ok": ([_int, _int, _int], _int),
    "btog_pass_workspace_bytes": ([_int, _i64, _i64, _int, _int], _sz),
    "btog_run_pass": ([_int, ctypes.POINTER(PassArgs), _int, _int, _ptr, _sz, _ptr], _int),
    "btog_last_error": ([], ctypes.c_char_p),
}
EXPORTS = tuple(_SIGS)

_loaded: dict = {}


class Library:
    """A generated library loaded through its C interface."""

    def __init__(self, path: str):
        self.path = path
        self.lib = ctypes.CDLL(path)
        for name, (args, res) in _SIGS.items():
            f = getattr(self.lib, name)
            f.argtypes = args
            f.restype = res
        if self.lib.btog_abi_version() != ABI_VERSION:
            raise ImportError(f"{path}: interface version {self.lib.btog_abi_version()}")

    def layout(self, k: int) -> tuple:
        c = (_int * 4)()
        self._check(self.lib.btog_pass_layout(k, c))
        return tuple(c)

    def config_ok(self, k: int, shape: int, rb: int) -> bool:
        return bool(self.lib.btog_config_ok(k, shape, rb))

    def workspace_bytes(self, k: int, m: int, n: int, shape: int, rb: int) -> int:
        return int(self.lib.btog_pass_workspace_bytes(k, m, n, shape, rb))

    def _check(self, status: int) -> None:
        if status != 0:
            from . import bto
            raise bto.BtoError(status, self.lib.btog_last_error().decode())


def load(prog: Program) -> Library:
    """The built library of `prog` (ImportError when it has not been built:
    there is no fallback)."""
    path = library_path(prog)
    if path not in _loaded:
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built: run btoc_gen.build (or the package build)")
        _loaded[path] = Library(path)
    return _loaded[path]


#: genomes found by the search (``tune``) on MI355X, keyed by program name,
#: used while the program's emitted source is unchanged.  BTO_GEN_TUNING
#: names another table of the same form.
TUNED_TABLE = os.path.join(PKG, "gen_tuned.json")


def tuned_table() -> dict:
    import json

    path = os.environ.get("BTO_GEN_TUNING") or TUNED_TABLE
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def tuned_genome(prog: Program) -> list | None:
    """The searched genome of `prog` when the table has one for its current
    source (same digest), else None."""
    ent = tuned_table().get(prog.name)
    if not ent or ent.get("digest") != digest(emit(prog)):
        return None
    return [tuple(g) for g in ent["genome"]]


def default_genome(prog: Program) -> list:
    """(shape, rb) per pass: the searched genome when the tuned table has
    one for this source; otherwise the sweep that stores an update in
    narrow tiles of short bands (as GEMVER's first pass in the library),
    sweeps that only read (contracted updates formed in registers included)
    with column sums in wide 4 x 4-wave tiles of 128 rows, and with row dots
    only in 2048-column tiles of 4 rows."""
    tuned = tuned_genome(prog)
    if tuned is not None and len(tuned) == len(gen_passes(prog)):
        return tuned
    return heuristic_genome(prog)


def heuristic_genome(prog: Program) -> list:
    """The genome chosen from each pass's structure alone."""
    out = []
    for p in gen_passes(prog):
        R, store, P, Q = layout(p)
        if store:
            out.append((0, 32))
        elif Q:
            out.append((6, 128))
        else:
            out.append((4, 4))
    return out


def genome_choices(prog: Program, lib: Library | None = None) -> list:
    """Every (shape, rb) each pass may take."""
    passes = gen_passes(prog)
    out = []
    for k, p in enumerate(passes):
        P = layout(p)[2]
        ok = []
        for s, (_, _, _, wr) in enumerate(SHAPES):
            for rb in RB_CHOICES:
                if rb % wr == 0 and rb >= wr and (not P or rb // wr <= 64):
                    ok.append((s, rb))
        out.append(ok)
    return out


def tune(prog: Program, bound: dict, reps: int = 5, warmup: int = 2, population: int = 20,
         generations: int = 6, seed: int = 0, log=None) -> dict:
    """Search the genome of `prog` on the bound inputs with the MFGA of
    Section IV (tune.mfga_genes), starting from the structural genome.  The
    fitness of a genome is the program's time on the device (HIP events on
    the current stream, `reps` runs after `warmup`); a genome whose outputs
    differ from the structural genome's by more than 1e-12 (normwise per
    output), or that the library refuses, scores infinity.  Returns the
    best genome, its time, the start's time and the number measured."""
    import torch

    from . import bto, tune as tuner

    start = heuristic_genome(prog)
    bound = dict(bound)
    first = run(prog, bound, start)
    torch.cuda.synchronize()
    bound.update(first)                      # later runs write the same tensors
    ref = [first[o].clone() for o in prog.outputs]
    choices = genome_choices(prog)

    def fitness(genome):
        try:
            for o in prog.outputs:
                bound[o].fill_(float("nan"))
            for _ in range(warmup):
                run(prog, bound, genome)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                run(prog, bound, genome)
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b) / reps
        except (bto.BtoError, SpecError):
            return float("inf")
        ok = tuner.outputs_agree([bound[o] for o in prog.outputs], ref)
        if log:
            log({"genome": [list(g) for g in genome], "ms": round(ms, 4), "checked": ok})
        return ms if ok else float("inf")

    t0 = fitness(tuple(start))
    best, ms, evals = tuner.mfga_genes(choices, fitness, start=start, population=population,
                                       generations=generations, seed=seed)
    return {"genome": [list(g) for g in best], "ms": ms, "start_ms": t0, "evaluations": evals}


def run(prog: Program, bound: dict, genome=None, ws=None) -> dict:
    """Enqueue the program on the current stream: its matrix passes in the
    generated library, its vector statements through libbto (see
    btoc_run.run for the binding rules).  `genome`: (shape, rb) per pass
    (default_genome when None)."""
    from . import btoc_run

    lib = load(prog)
    passes = gen_passes(prog)
    genome = default_genome(prog) if genome is None else list(genome)
    if len(genome) != len(passes):
        raise SpecError(f"genome has {len(genome)} entries for {len(passes)} passes")
    return btoc_run.run(prog, bound, ws, gen=(lib, passes, genome))


def synthetic_bound(prog: Program, n: int, dev, seed_base: int = 970) -> dict:
    """Seeded uniform[-1, 1) inputs of an n x n instance of `prog` on `dev`
    (scalars 1.5, 0.7, ... in declaration order); column-major matrices as
    transposed views of row-major storage."""
    import torch

    from . import bto, synth

    bound = {}
    scal = iter((1.5, 0.7, 1.25, 0.5, 2.0, 0.3, 1.1, 0.9))
    for j, name in enumerate(prog.inputs):
        kind = prog.kinds[name]
        sid = synth.stream_id(13, seed_base + j)
        if kind == "scalar":
            bound[name] = next(scal)
        elif kind == "matrix":
            A = torch.empty((n, n), dtype=torch.float64, device=dev)
            bto.synth_fill(A, synth.stream_state(synth.SEED, sid))
            bound[name] = A.t() if name in prog.colmajor else A
        else:
            v = torch.empty(n, dtype=torch.float64, device=dev)
            bto.synth_fill(v, synth.stream_state(synth.SEED, sid))
            bound[name] = v
    return bound


def alg_bytes(prog: Program, m: int, n: int) -> int:
    """Algorithmic HBM bytes of the program's generated schedule: each pass
    reads its matrix once and writes a stored update once; each vector a
    pass reads or writes counts once per pass."""
    total = 0
    for p in gen_passes(prog):
        R, store, P, Q = layout(p)
        total += m * n * 8 * (2 if store else 1)
        vec = R * (m + n) + P * (n + m) + Q * (m + n)
        vec += sum(m for r in p.rows if r.get("add") is not None)
        vec += sum(n for c in p.cols if c.get("add") is not None)
        total += 8 * vec
    return total


def _tune_main(names, n, table_path) -> int:
    import json
    import time

    import torch

    from . import bto_specs, tune as tuner

    dev = torch.device("cuda:0")
    table = {}
    if os.path.exists(table_path):
        with open(table_path) as f:
            table = json.load(f)
    for name in names:
        prog = compile_spec(bto_specs.GENERATED[name], target="generated")
        bound = synthetic_bound(prog, n, dev)
        t0 = time.perf_counter()
        res = tune(prog, bound, log=lambda r: print(json.dumps({name: r}), flush=True))
        res.update({"digest": digest(emit(prog)), "n": n,
                    "environment": tuner.environment_key(digest=digest(emit(prog))),
                    "search_s": round(time.perf_counter() - t0, 1)})
        table[prog.name] = res
        print(json.dumps({prog.name: res}), flush=True)
        del bound
        torch.cuda.empty_cache()
    with open(table_path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    # run as the package's module, so that its ctypes types are the ones
    # the runtime (btoc_run) builds
    from paper_1205_1098_amd.btoc_gen import main as _main

    raise SystemExit(_main())
