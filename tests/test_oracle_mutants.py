"""Planted mistakes in the oracle (CPU only).

Each entry edits one spot of a copy of the oracle's C source the way a
plausible slip would: a dropped term, a wrong sign, bound or index, a transposed
operand, a misread constant.  The copy is built on the side and the CPU pin
modules named with it run against it in a child process; every copy must fail
at least one of them.  A mutant that passes them all marks a gap in the pins.
The committed oracle is never touched: the copies exist only in the test's
temporary directory.
"""
import json
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_DIR = os.path.join(ROOT, "oracle")

RNG, GOLD, GRU, CNN, DYN, MET, PAP, REG = ("test_oracle_rng.py", "test_golden.py", "test_oracle_controller.py",
                                           "test_oracle_cnn.py", "test_oracle_dynamics.py", "test_oracle_metrics.py",
                                           "test_oracle_paper.py", "test_oracle_regrowth.py")

# name -> (text in oracle.c, its replacement, occurrences replaced, the pin modules expected to catch it)
MUTANTS = {
    # random primitives
    "philox_nine_rounds": ("round < 10; ++round", "round < 9; ++round", 1, (GOLD, RNG)),
    "philox_weyl_constant": ("k1 += 0xBB67AE85u;", "k1 += 0xBB67AE87u;", 1, (GOLD, RNG)),
    "counter_entity_step_swapped": ("philox_block(entity, step, stream, block, (uint32_t)seed, (uint32_t)(seed >> 32), out);",
                                    "philox_block(step, entity, stream, block, (uint32_t)seed, (uint32_t)(seed >> 32), out);",
                                    1, (DYN,)),
    "ln_series_coefficient": ("r = fmaf(r, s2, 2.0f / 5.0f);", "r = fmaf(r, s2, 2.0f / 6.0f);", 1, (RNG,)),
    "ln_correction_sign": ("return fmaf(ef, 0x1.62e4p-1f, f - corr);", "return fmaf(ef, 0x1.62e4p-1f, f + corr);", 1,
                           (RNG,)),
    "cos_series_sign": ("p = fmaf(p, x2, -1.0f / 720.0f);", "p = fmaf(p, x2, 1.0f / 720.0f);", 1, (RNG,)),
    "quadrant_rotation_sign": ("    case 1: *s_out = cf;  *c_out = -sf; break;", "    case 1: *s_out = cf;  *c_out = sf; break;",
                               1, (RNG,)),
    "gauss_radius_without_2": ("sqrtf(-2.0f * ln_unit(u1))", "sqrtf(-ln_unit(u1))", 1, (RNG,)),
    "gauss_sin_cos_swapped": ("*z0 = r * c;\n    *z1 = r * s;", "*z0 = r * s;\n    *z1 = r * c;", 1, (RNG,)),
    "gumbel_sign": ("    return -ln_unit(e);", "    return ln_unit(e);", 1, (CNN,)),
    "gumbel_uniform_offset": ("(float)(((word >> 9) << 1) | 1u) * 0x1p-24f", "(float)(word >> 8) * 0x1p-24f", 1, (CNN,)),
    # the GRU controller and its initial genome
    "gru_reset_dropped": ("tanh(gi[2] + r * gh[2])", "tanh(gi[2] + gh[2])", 1, (GRU,)),
    "gru_update_convention": ("(1.0 - z) * n + z * (double)h[k]", "z * n + (1.0 - z) * (double)h[k]", 1, (GRU,)),
    "gru_w_hh_transposed": ("th[L.hh + (j * hd + k) * 3 + g]", "th[L.hh + (k * hd + j) * 3 + g]", 1, (GRU,)),
    "gru_update_gate_copy": ("double z = sigmoid(gi[1] + gh[1]);", "double z = sigmoid(gi[0] + gh[0]);", 1, (GRU,)),
    "gru_head_transposed": ("s += (double)th[L.wo + a * hd + k] * h_out[k];", "s += (double)th[L.wo + k * 5 + a] * h_out[k];",
                            1, (GRU,)),
    "gru_head_bias_dropped": ("double s = (double)th[L.bo + a];", "double s = 0.0;", 1, (GRU,)),
    "init_biases_random": ("else if (p < L->wo) std = 0.0f;", "else if (p < L->wo) std = std_hd;", 1, (GRU,)),
    "init_std_over_fan_in": ("float std_ih = (float)(w->cfg.w_init_gain / sqrt((double)L->n_in));",
                             "float std_ih = (float)(w->cfg.w_init_gain / (double)L->n_in);", 1, (GRU,)),
    # observation
    "observe_window_transposed": ("int k = (dy + rho) * win + (dx + rho);", "int k = (dx + rho) * win + (dy + rho);", 1,
                                  (GRU,)),
    "observe_outside_free": ("                x[win * win + k] = 1.0;", "                x[win * win + k] = 0.0;", 1,
                             (GRU,)),
    "observe_own_cell_free": ("x[win * win + k] = (w->cnt[r * W + c] > 0) ? 1.0 : 0.0;",
                              "x[win * win + k] = (w->cnt[r * W + c] > 0 && (dy || dx)) ? 1.0 : 0.0;", 1, (GRU,)),
    "observe_energy_scale": ("x[2 * win * win] = (double)w->e[a] / (double)w->cfg.E0;",
                             "x[2 * win * win] = (double)w->e[a];", 1, (GRU,)),
    # the paper's network and its sampling
    "cnn_kernel_transposed": ("th[L.c1w + ((ky * CNN_K + kx) * CNN_CH + ci) * CNN_F1 + co]",
                              "th[L.c1w + ((kx * CNN_K + ky) * CNN_CH + ci) * CNN_F1 + co]", 1, (CNN,)),
    "cnn_padding_dropped": ("int iy = oy * CNN_S + ky - L.pad1, ix = ox * CNN_S + kx - L.pad1;",
                            "int iy = oy * CNN_S + ky, ix = ox * CNN_S + kx;", 1, (CNN,)),
    "cnn_conv2_padding_dropped": ("int iy = oy * CNN_S + ky - L.pad2, ix = ox * CNN_S + kx - L.pad2;",
                                  "int iy = oy * CNN_S + ky, ix = ox * CNN_S + kx;", 1, (CNN,)),
    "observe_cnn_channels_swapped": ("px[0] = w->R[r * W + c] ? 1.0 : 0.0;", "px[1] = w->R[r * W + c] ? 1.0 : 0.0;", 1,
                                     (CNN,)),
    "sampling_fifth_word_reused": ("float g = gumbel_of_word(a < 4 ? r0[a] : r1[a - 4]);",
                                   "float g = gumbel_of_word(r0[a % 4]);", 1, (CNN,)),
    "cnn_pool_sum": ("q1[(y * L.p1 + x) * CNN_F1 + ch] = s / (double)(CNN_POOL * CNN_POOL);",
                     "q1[(y * L.p1 + x) * CNN_F1 + ch] = s;", 1, (CNN,)),
    "lstm_input_forget_swapped": ("c_out[k] = fg * (double)c[k] + ig * gg;", "c_out[k] = ig * (double)c[k] + fg * gg;",
                                  1, (CNN,)),
    "lstm_bias_dropped": ("double s = (double)th[L.lb + g * CNN_HD + k];", "double s = 0.0;", 1, (CNN,)),
    "dense8_reads_cell_state": ("cat[L.emb + k] = h_out[k];", "cat[L.emb + k] = c_out[k];", 1, (CNN,)),
    "ate_bit_dropped": ("emb[L.flat + CNN_NA] = ate ? 1.0 : 0.0;", "emb[L.flat + CNN_NA] = 0.0;", 1, (CNN,)),
    "cnn_init_lstm_fan": ("else if (p < L.lb) fan = CNN_HD;", "else if (p < L.lb) fan = L.emb;", 1, (CNN,)),
    "cnn_init_dense_fan": ("else if (p < L.d8b) fan = L.cat;", "else if (p < L.d8b) fan = CNN_D;", 1, (CNN,)),
    "dense5_transposed": ("s += (double)th[L.d5w + o * CNN_NA + a] * y8[o];", "s += (double)th[L.d5w + a * CNN_D + o] * y8[o];",
                          1, (CNN,)),
    "dense8_without_tanh": ("y8[o] = tanh(s);", "y8[o] = s;", 1, (CNN,)),
    "prev_action_one_hot_shifted": ("emb[L.flat + a] = (prev_action == a) ? 1.0 : 0.0;",
                                    "emb[L.flat + a] = (prev_action == a + 1) ? 1.0 : 0.0;", 1, (CNN,)),
    "prev_action_before_resync": ("w->pact[a] = act;", "w->pact[a] = best;", 1, (CNN,)),
    "temperature_inverted": ("float sc = 50.0f * lf[a];", "float sc = lf[a] / 50.0f;", 1, (CNN,)),
    "observe_cnn_wall_channel": ("                px[2] = 1.0;", "                px[2] = 0.0;", 1, (CNN,)),
    # benchmark dynamics
    "move_into_occupied": ("            if (w->occ[cell] != -1) continue;\n", "", 1, (DYN,)),
    "east_west_swapped": ("static const int DC[5] = {0, 0, 1, -1, 0};", "static const int DC[5] = {0, 0, -1, 1, 0};", 1,
                          (DYN,)),
    "moves_see_earlier_moves": ("            if (w->occ[cell] != -1) continue;\n            uint32_t rr[4];",
                                "            if (w->occ[cell] != -1 || w->who[cell] != -1) continue;\n            uint32_t rr[4];",
                                1, (DYN,)),
    "energy_decay_only_unfed": ("w->e[a] = w->e[a] - cfg->decay + cfg->gain * (int32_t)w->ate[a];",
                                "w->e[a] = w->e[a] + (w->ate[a] ? cfg->gain : -cfg->decay);", 1, (DYN,)),
    "death_age_bound": ("(w->age[a] >= cfg->L_max)", "(w->age[a] > cfg->L_max)", 1, (DYN,)),
    "death_energy_bound": ("(w->e[a] <= 0)", "(w->e[a] < 0)", 1, (DYN,)),
    "streak_not_reset": ("            w->streak[a] = 0;\n            w->occ[w->claim[a]] = c;",
                         "            w->occ[w->claim[a]] = c;", 1, (DYN,)),
    "streak_strict_threshold": ("w->streak[a] = (w->e[a] >= cfg->E_repr) ? w->streak[a] + 1 : 0;",
                                "w->streak[a] = (w->e[a] > cfg->E_repr) ? w->streak[a] + 1 : 0;", 1, (DYN,)),
    "child_in_current_window": ("w->wvalid[c] = 0;   /* not alive", "w->wvalid[c] = 1;   /* not alive", 1, (MET,)),
    "birth_start_direction": ("int d0 = (int)(rr[0] & 3u);", "int d0 = 0;", 1, (DYN,)),
    "move_draw_stream": ("draw(w->seed, w->uid[a], t, ORACLE_S_MOVE, 0, rr);",
                         "draw(w->seed, w->uid[a], t, ORACLE_S_BIRTH, 0, rr);", 1, (DYN,)),
    "child_energy": ("w->e[c] = cfg->E0;", "w->e[c] = w->e[a];", 2, (DYN,)),
    "mutation_keyed_by_parent": ("draw(w->seed, cu, t, ORACLE_S_MUTATE", "draw(w->seed, w->uid[a], t, ORACLE_S_MUTATE",
                                 2, (DYN,)),
    "mutation_sigma_doubled": ("float sigma = (float)cfg->sigma_mut;", "float sigma = 2.0f * (float)cfg->sigma_mut;", 2,
                               (DYN,)),
    # the initial world
    "placement_highest_draws": ("uint32_t cell = (uint32_t)(keys[a] & 0xFFFFFFFFu);",
                                "uint32_t cell = (uint32_t)(keys[HW - 1 - (size_t)a] & 0xFFFFFFFFu);", 1, (DYN, REG)),
    "resources_from_placement_stream": ("draw(seed, (uint32_t)i, 0, ORACLE_S_INIT_RES, 0, r);",
                                        "draw(seed, (uint32_t)i, 0, ORACLE_S_INIT_PLACE, 0, r);", 1, (DYN, REG)),
    "birth_claim_same_word": ("uint64_t key = claim_key(rr[1], w->uid[a]);", "uint64_t key = claim_key(rr[0], w->uid[a]);",
                              1, (DYN,)),
    # compaction of the survivors (both rule sets)
    "compaction_drops_previous_action": ("            w->pact[n_surv] = w->pact[a];\n", "", 2, (CNN, DYN, PAP)),
    "compaction_drops_streak": ("            w->streak[n_surv] = w->streak[a];\n", "", 2, (CNN, DYN, PAP)),
    "compaction_drops_window_start": ("            w->wrow[n_surv] = w->wrow[a];\n", "", 2, (MET,)),
    "compaction_drops_ate_bit": ("            w->pate[n_surv] = w->pate[a];\n", "", 2, (CNN, DYN, PAP)),
    "compaction_drops_hidden_state": (
        "            memmove(w->h + (size_t)n_surv * hd, w->h + (size_t)a * hd, (size_t)hd * sizeof(float));\n", "", 2,
        (GRU, CNN, DYN, PAP)),
    "compaction_drops_genome": (
        "            memmove(w->theta + (size_t)n_surv * P, w->theta + (size_t)a * P, P * sizeof(float));\n", "", 2,
        (GRU, CNN, DYN, PAP)),
    "compaction_drops_age": ("            w->age[n_surv] = w->age[a];\n", "", 2, (CNN, DYN, PAP, MET)),
    "compaction_drops_window_flag": ("            w->wvalid[n_surv] = w->wvalid[a];\n", "", 2, (MET,)),
    "slots_one_short": ("int free_slots = cfg->cap - w->n;", "int free_slots = cfg->cap - w->n - 1;", 2, (DYN, PAP)),
    "claims_when_full": ("if (free_slots <= 0 || w->streak[a] < cfg->T_repr) continue;",
                         "if (w->streak[a] < cfg->T_repr) continue;", 1, (DYN,)),
    # regrowth
    "regrowth_latitude_flipped": ("double a = d * (double)row;", "double a = d * (double)(cfg->H - 1 - row);", 1,
                                  (REG,)),
    "threshold_rounded_up": ("return (uint64_t)floor(p * 4294967296.0);", "return (uint64_t)ceil(p * 4294967296.0);",
                             1, (REG,)),
    "regrowth_spontaneous_dropped": ("double p = q + cfg->spont;", "double p = q;", 1, (REG,)),
    "regrowth_neighbourhood_short": (
        "for (int dy = -2; dy <= 2; ++dy)\n                    for (int dx = -2; dx <= 2; ++dx)",
        "for (int dy = -2; dy <= 1; ++dy)\n                    for (int dx = -2; dx <= 2; ++dx)", 1, (REG,)),
    "regrowth_not_synchronous": ("if ((uint64_t)rr[0] < w->thr[r * 25 + n]) Rn[r * W + c] = 1;",
                                 "if ((uint64_t)rr[0] < w->thr[r * 25 + n]) Rn[r * W + c] = w->R[r * W + c] = 1;", 1,
                                 (REG, PAP)),
    # the paper's dynamics
    "paper_climate_flipped": ("double x = (double)row / (double)(cfg->H - 1);",
                              "double x = 1.0 - (double)row / (double)(cfg->H - 1);", 1, (PAP,)),
    "paper_climate_denominator": ("double x = (double)row / (double)(cfg->H - 1);",
                                  "double x = (double)row / (double)cfg->H;", 1, (PAP,)),
    "paper_any_neighbour": ("double pI = (n == 1) ? cfg->regrow_pI : 0.0;",
                            "double pI = (n >= 1) ? cfg->regrow_pI : 0.0;", 1, (PAP,)),
    "paper_no_energy_clip": ("        if (e > cfg->E_max) e = cfg->E_max;\n", "", 1, (PAP,)),
    "paper_walls_block": ("            w->walldead[a] = 1;\n", "", 1, (PAP,)),
    "paper_death_streak_bound": ("(-s >= cfg->T_death)", "(-s > cfg->T_death)", 1, (PAP,)),
    "paper_agent_channel_binary": ("px[1] = (double)w->cnt[r * W + c];", "px[1] = w->cnt[r * W + c] > 0 ? 1.0 : 0.0;",
                                   1, (PAP,)),
    "paper_eat_draw_stream": ("draw(w->seed, w->uid[a], t, ORACLE_S_EAT, 0, rr);",
                              "draw(w->seed, w->uid[a], t, ORACLE_S_MOVE, 0, rr);", 1, (PAP,)),
    "paper_wall_dead_eats": ("        if (w->walldead[a]) continue;\n", "", 1, (PAP,)),
    "paper_dead_age_off_by_one": ("inf->dead_age += w->age[a];", "inf->dead_age += w->age[a] - 1;", 1, (PAP, MET)),
    "paper_streak_at_threshold": ("if (e > cfg->E_repr) s = (s > 0 ? s : 0) + 1;",
                                  "if (e >= cfg->E_repr) s = (s > 0 ? s : 0) + 1;", 1, (PAP,)),
    "paper_death_at_threshold": ("else if (e < cfg->E_repr) s = (s < 0 ? s : 0) - 1;",
                                 "else if (e <= cfg->E_repr) s = (s < 0 ? s : 0) - 1;", 1, (PAP,)),
    "paper_age_bound": ("(w->age[a] > cfg->L_max)", "(w->age[a] >= cfg->L_max)", 1, (PAP,)),
    "paper_slots_one_short": ("    int free_slots = cfg->cap - w->n;\n    inf->claim_wins",
                              "    int free_slots = cfg->cap - w->n - 1;\n    inf->claim_wins", 1, (PAP,)),
    "paper_eat_without_resource": ("        if (!w->R[cell]) continue;\n", "", 1, (PAP,)),
    "paper_parent_streak_kept": ("        w->streak[a] = 0;\n        w->n++;", "        w->n++;", 1, (PAP,)),
    # ecology metrics and the lab's greediness
    "move_metric_chebyshev": ("int dist = abs(w->row[a] - w->wrow[a]) + abs(w->col[a] - w->wcol[a]);",
                              "int dist = abs(w->row[a] - w->wrow[a]) > abs(w->col[a] - w->wcol[a]) ? "
                              "abs(w->row[a] - w->wrow[a]) : abs(w->col[a] - w->wcol[a]);", 1, (MET,)),
    "move_metric_bin_width": ("hist[dist / 3]++;", "hist[dist / 4]++;", 1, (MET,)),
    "move_window_start": ("if (w->t % ORACLE_MOVE_WINDOW == 0) {", "if (w->t % ORACLE_MOVE_WINDOW == 1) {", 1, (MET,)),
    "dead_age_off_by_one": ("inf.dead_age += w->age[a];   /*", "inf.dead_age += w->age[a] - 1;   /*", 1, (MET,)),
    "seen_window_short": ("for (int dy = -w->rho; dy <= w->rho && !sees; ++dy)",
                          "for (int dy = -w->rho; dy < w->rho && !sees; ++dy)", 1, (MET,)),
}


def run_mutant(name, tmp):
    old, new, count, pins = MUTANTS[name]
    src = open(os.path.join(ORACLE_DIR, "oracle.c")).read()
    assert src.count(old) == count, (name, src.count(old))
    d = os.path.join(tmp, name)
    os.makedirs(d)
    shutil.copy(os.path.join(ORACLE_DIR, "oracle.h"), d)
    with open(os.path.join(d, "oracle.c"), "w") as f:
        f.write(src.replace(old, new))
    env = dict(os.environ, ORACLE_SRC=os.path.join(d, "oracle.c"), ORACLE_LIB=os.path.join(d, "liboracle.so"))
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu and not slow", "-p", "no:cacheprovider",
           *[os.path.join(HERE, p) for p in pins]]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    failed = [ln.split()[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED ")]
    return r.returncode, failed, r.stdout[-2000:] + r.stderr[-2000:]


def run_all(tmp):
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        futs = {n: ex.submit(run_mutant, n, tmp) for n in MUTANTS}
        return {n: f.result() for n, f in futs.items()}


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    run_uid = os.environ.get("PYTEST_XDIST_TESTRUNUID")
    if not run_uid:
        return run_all(str(tmp_path_factory.mktemp("mutants")))
    # Under pytest-xdist each worker that draws one of these tests would run
    # every mutant again: the first worker runs them and the others of the
    # same test run read its results.
    from filelock import FileLock
    out = tmp_path_factory.getbasetemp().parent / f"mutants-{run_uid}.json"
    with FileLock(str(out) + ".lock"):
        if out.exists():
            return {n: tuple(v) for n, v in json.loads(out.read_text()).items()}
        res = run_all(str(tmp_path_factory.mktemp("mutants")))
        out.write_text(json.dumps(res))
        return res


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_is_caught(results, name):
    rc, failed, tail = results[name]
    assert rc == 1 and failed, f"{name}: no pin failed (exit {rc})\n{tail}"
    print(f"{name}: caught by {failed[0]}")
