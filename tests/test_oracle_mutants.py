"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (a flipped sign, a
dropped term, a transposed operand, a wrong index or tie-break, a wrong
stopping rule), builds it on the CPU and runs the pin suites against it with
``LEIDEN_ORACLE_LIB``; at least one pin has to fail.  The committed oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "leiden_oracle.cpp")

# (name, text in the oracle, replacement)
MUTANTS = [
    ("eq2_sign", "  return first - second;\n}", "  return first + second;\n}"),
    ("eq2_transposed_sigma", "double b = (double)(Ki + Sc - Sd);", "double b = (double)(Ki + Sd - Sc);"),
    ("eq2_drop_kid", "double a = (double)(Kic - Kid);", "double a = (double)(Kic);"),
    ("scan_keeps_self_loop", "    if (!self && j == i) continue;\n    H.add(C[j], G.w[e]);\n  }\n  return",
     "    H.add(C[j], G.w[e]);\n  }\n  return"),
    ("tie_break_highest", "if (!best.found || dq > best.dq || (dq == best.dq && c < best.c)) {\n      best.found = true;\n      best.c = c;\n      best.dq = dq;\n    }\n  }\n  return best;",
     "if (!best.found || dq > best.dq || (dq == best.dq && c > best.c)) {\n      best.found = true;\n      best.c = c;\n      best.dq = dq;\n    }\n  }\n  return best;"),
    ("move_on_nonpositive", "      if (!ch.found || !(ch.dq > 0.0)) continue;\n      L.S[d] -= L.K[i];",
     "      if (!ch.found || !(ch.dq > -1.0)) continue;\n      L.S[d] -= L.K[i];"),
    ("q_sigma_all_edges", "if (C[i] == C[G.cols[e]]) p.sigma += w;", "p.sigma += w;"),
    ("q_no_square", "p.T += (u128)(u64)Sig[c] * (u128)(u64)Sig[c];", "p.T += (u128)(u64)Sig[c];"),
    ("aggregate_drops_self", "for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) t.emplace_back(C[i], C[G.cols[e]], G.w[e]);",
     "for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) if (C[i] != C[G.cols[e]]) t.emplace_back(C[i], C[G.cols[e]], G.w[e]);"),
    ("renumber_max_member", "    if (rep[c] == kEmpty) rep[c] = i;", "    rep[c] = i;"),
    ("split_no_grouping", "      out[u] = s;", "      out[u] = u;"),
    ("refine_unbounded", "    if (CB[i] != CB[j]) continue;\n", ""),
    ("update_weights_sign", "  for (const Entry& x : dels) {\n    K[x.i] -= x.w;", "  for (const Entry& x : dels) {\n    K[x.i] += x.w;"),
    ("refine_threshold_flipped", "* o.tau_re_den > (u128)", "* o.tau_re_den < (u128)"),
    ("delta_sigma_no_reset", "    if (P.dR[c]) dSig[c] = 0;", "    if (P.dR[c] && false) dSig[c] = 0;"),
    ("df_insertion_condition", "    for (const Entry& x : inss)\n      if (Cp[x.i] != Cp[x.j]) dV[x.i] = 1;",
     "    for (const Entry& x : inss)\n      if (Cp[x.i] == Cp[x.j]) dV[x.i] = 1;"),
    ("track_min_overlap", "    if (it == best_of_old.end() || w > it->second.second ||", "    if (it == best_of_old.end() || w < it->second.second ||"),
    ("static_labels_unordered", "    if (id[C[i]] == kEmpty) id[C[i]] = next++;\n    out[i] = id[C[i]];",
     "    if (id[C[i]] == kEmpty) id[C[i]] = next++;\n    out[i] = C[i];"),
    ("row_sums_unweighted", "    for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) K[i] += G.w[e];", "    for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) K[i] += 1;"),
    ("ds_mark_dropped", "      if (dE[i])\n        for (i64 e = G.offs[i]; e < G.offs[i + 1]; ++e) dV[G.cols[e]] = 1;", ""),
    # convergence control (Alg. 4, Alg. 6)
    ("seq_stop_strict", "      if (dynamic) L.dS[d] = 1;\n    }\n    r.iterations = li + 1;\n    if (fixed_to_gain(dQ) <= tau) break;",
     "      if (dynamic) L.dS[d] = 1;\n    }\n    r.iterations = li + 1;\n    if (fixed_to_gain(dQ) < tau) break;"),
    ("jacobi_stop_strict", "        }\n      }\n    }\n    r.iterations = li + 1;\n    if (fixed_to_gain(dQ) <= tau) break;",
     "        }\n      }\n    }\n    r.iterations = li + 1;\n    if (fixed_to_gain(dQ) < tau) break;"),
    ("iterations_zero_based", "    r.iterations = li + 1;", "    r.iterations = li;"),
    ("no_tau_decline", "    tau = tau / (double)o.tol_decline;\n", ""),
    ("final_lookup_unrefined", "  for (u32 v = 0; v < n; ++v) C[v] = L.C[C[v]];\n  return C;",
     "  for (u32 v = 0; v < n; ++v) C[v] = CB[C[v]];\n  return C;"),
    ("pass_break_ignores_refined", "    if (li <= 1 && !refined) break;", "    if (li <= 1) break;"),
    ("pass_break_never_later", "    if (li <= 1 && lp > 0) break;\n", ""),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: " + name
    mutated = src.replace(old, new, 1)
    cpp = tmp_path / "mutant.cpp"
    lib = tmp_path / "libmutant.so"
    cpp.write_text(mutated)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-ffp-contract=off", "-shared", "-fPIC", "-o", str(lib),
                           str(cpp)])
    env = dict(os.environ, LEIDEN_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_convergence.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutant %s:\n%s" % (name, r.stdout[-2000:])
