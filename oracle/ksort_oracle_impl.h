/*
 * K-sort CPU oracle, type-generic body -- TEST INFRASTRUCTURE ONLY.
 *
 * Included twice by ksort_oracle.c, once with KEY_T = double and once with
 * KEY_T = float; SFX(name) appends the type suffix.  Every function follows
 * arXiv 1107.3622, Section 1.1, in the paper's own order and names.
 *
 * Readings of the text used here (each one is a choice where the text is
 * silent or self-contradictory):
 *   R1  Step-2's loop condition on the gap between j and i is read as a
 *       loop that runs while j - i >= 2.  The illustration (Section 1.2,
 *       first row) needs the comparison made at j - i == 2.
 *   R2  `flag` is never initialised in Step-1; it is cleared on every
 *       partition entry.  The third illustration row shows "Temp = Nil".
 *   R3  Indices are 0-based: the whole array is a[0..n-1].
 *   R4  Step-5's left side runs from the segment's first position up to
 *       the key's final index, the key excluded: [left, i-1], processed when
 *       left < i-1 (at least two elements; the Section 1.2 note says a
 *       single value needs no processing).
 *   R5  Step-6's printed test compares left with i+1 and can never hold,
 *       because i >= left; it is read as right > i+1 on [i+1, right], the
 *       mirror of Step-5.  The illustration goes on to process the right
 *       side.
 *   R6  Sub-arrays are processed depth-first, left side first, the row order
 *       of the illustration.  Only the order of trace records depends on it.
 *   R7  The comparison is exactly `key <= a[p]` in KEY_T: ties go right, and
 *       a NaN compares false and so goes left.
 */

/* Steps 1-4: partition a[left..right] around key = a[left]. */
int64_t SFX(ksort_oracle_partition)(KEY_T *a, int64_t left, int64_t right,
                                    ksort_oracle_call *rec)
{
    /* Step-1: the first element is the key; i = left, j = right + 1,
     * p = left + 1 and k = p.  flag starts cleared (R2). */
    KEY_T key = a[left];
    KEY_T temp = 0;
    int flag = 0;
    int64_t i = left;
    int64_t j = right + 1;
    int64_t p = left + 1;
    int64_t k = p;
    int64_t comparisons = 0;

    /* Step-2: repeat Step-3 while j - i >= 2 (R1). */
    while (j - i >= 2) {
        comparisons++;
        /* Step-3: compare a[p] with the key. */
        if (key <= a[p]) {
            /* Step-3.1 */
            if (p != j && j != right + 1) {
                a[j] = a[p];
            } else if (j == right + 1) {
                temp = a[p];
                flag = 1;
            }
            j = j - 1;
            p = j;
        } else {
            /* Step-3.2 (key > a[p]) */
            a[i] = a[p];
            i = i + 1;
            k = k + 1;
            p = k;
        }
    }

    /* Step-4: the key goes to a[i]; temp, if one was taken, to a[i+1]. */
    a[i] = key;
    if (flag == 1)
        a[i + 1] = temp;

    if (rec) {
        rec->left = left;
        rec->right = right;
        rec->i = i;
        rec->comparisons = comparisons;
        rec->k_minus_i = k - i;
        rec->key = (double)key;
        rec->temp = flag ? (double)temp : 0.0;
        rec->flag = flag;
        rec->pad = 0;
    }
    return i;
}

/* Steps 1-6 on a[0..n-1] with an explicit stack of pending sub-arrays, so
 * that the worst-case depth (n, for sorted input) cannot overflow the C
 * stack.  The right side is pushed first so that the left side is popped
 * first (R6). */
int SFX(ksort_oracle_sort)(KEY_T *a, int64_t n, int64_t *first_pivot,
                           ksort_oracle_call *trace, int64_t trace_cap,
                           int64_t *ncalls, int64_t *ncomparisons)
{
    int64_t calls = 0, comps = 0;
    if (first_pivot)
        *first_pivot = (n == 0) ? -1 : 0;
    if (n >= 2) {
        int64_t cap = 64, top = 0;
        int64_t *stk = (int64_t *)malloc((size_t)cap * 2 * sizeof(int64_t));
        if (!stk)
            return -2;
        stk[0] = 0;
        stk[1] = n - 1;
        top = 1;
        while (top > 0) {
            top--;
            int64_t left = stk[2 * top], right = stk[2 * top + 1];
            ksort_oracle_call rec;
            int64_t i = SFX(ksort_oracle_partition)(a, left, right, &rec);
            if (calls == 0 && first_pivot)
                *first_pivot = i;
            if (trace && calls < trace_cap)
                trace[calls] = rec;
            calls++;
            comps += rec.comparisons;
            if (top + 2 > cap) {
                int64_t ncap = cap * 2;
                int64_t *nstk = (int64_t *)realloc(stk, (size_t)ncap * 2 * sizeof(int64_t));
                if (!nstk) {
                    free(stk);
                    return -2;
                }
                stk = nstk;
                cap = ncap;
            }
            /* Step-6 (R5): the side right of the key, if it has two or more
             * elements. */
            if (right > i + 1) {
                stk[2 * top] = i + 1;
                stk[2 * top + 1] = right;
                top++;
            }
            /* Step-5 (R4): the side left of the key, if it has two or more
             * elements. */
            if (left < i - 1) {
                stk[2 * top] = left;
                stk[2 * top + 1] = i - 1;
                top++;
            }
        }
        free(stk);
    }
    if (ncalls)
        *ncalls = calls;
    if (ncomparisons)
        *ncomparisons = comps;
    return 0;
}

/* Steps 1-6 on a[0..n-1] by up to `threads` threads.  Every partition call
 * is the literal one (ksort_oracle_partition); only sub-arrays that share no
 * element run at the same time, so the final array equals the one-thread
 * run's.  The threads share one stack of pending sub-arrays: a thread pops
 * one, makes its call and pushes the sides of two or more elements (right
 * side first, so the left one is popped first), or finishes a sub-array of
 * at most `grain` elements alone with ksort_oracle_sort.  first_pivot as in
 * ksort_oracle_sort.  Returns 0, or -2 when memory or a thread cannot be had. */
struct SFX(oracle_pool) {
    KEY_T *a;
    int64_t n, grain;
    pthread_mutex_t mu;
    pthread_cond_t cv;
    int64_t *stk;       /* (left, right) pairs */
    int64_t top, cap;
    int64_t pending;    /* sub-arrays pushed and not yet done */
    int64_t *first_pivot;
    int rc;
};

/* Pushes [left, right] (caller holds the lock); 0 or -2. */
static int SFX(oracle_push)(struct SFX(oracle_pool) *q, int64_t left, int64_t right)
{
    if (q->top == q->cap) {
        int64_t *ns = (int64_t *)realloc(q->stk, (size_t)q->cap * 4 * sizeof(int64_t));
        if (!ns)
            return -2;
        q->stk = ns;
        q->cap *= 2;
    }
    q->stk[2 * q->top] = left;
    q->stk[2 * q->top + 1] = right;
    q->top++;
    q->pending++;
    return 0;
}

static void *SFX(oracle_worker)(void *arg)
{
    struct SFX(oracle_pool) *q = (struct SFX(oracle_pool) *)arg;
    pthread_mutex_lock(&q->mu);
    for (;;) {
        while (q->top == 0 && q->pending > 0 && q->rc == 0)
            pthread_cond_wait(&q->cv, &q->mu);
        if (q->top == 0 || q->rc != 0)
            break;  /* everything is done, or a failure stops the run */
        q->top--;
        const int64_t left = q->stk[2 * q->top], right = q->stk[2 * q->top + 1];
        pthread_mutex_unlock(&q->mu);
        int rc = 0;
        int64_t i = -1;
        if (right - left + 1 <= q->grain)
            rc = SFX(ksort_oracle_sort)(q->a + left, right - left + 1, NULL, NULL, 0, NULL, NULL);
        else
            i = SFX(ksort_oracle_partition)(q->a, left, right, NULL);
        pthread_mutex_lock(&q->mu);
        if (i >= 0) {
            if (left == 0 && right == q->n - 1 && q->first_pivot)
                *q->first_pivot = i;
            /* Step-6 (R5), then Step-5 (R4) */
            if (rc == 0 && right > i + 1)
                rc = SFX(oracle_push)(q, i + 1, right);
            if (rc == 0 && left < i - 1)
                rc = SFX(oracle_push)(q, left, i - 1);
        }
        if (rc != 0)
            q->rc = rc;
        q->pending--;
        pthread_cond_broadcast(&q->cv);
    }
    pthread_mutex_unlock(&q->mu);
    return NULL;
}

int SFX(ksort_oracle_sort_parallel)(KEY_T *a, int64_t n, int threads, int64_t *first_pivot)
{
    if (threads < 1)
        threads = 1;
    int64_t grain = n / (64 * (int64_t)threads);
    if (grain < 4096)
        grain = 4096;
    if (threads == 1 || n <= grain)
        return SFX(ksort_oracle_sort)(a, n, first_pivot, NULL, 0, NULL, NULL);
    struct SFX(oracle_pool) q;
    memset(&q, 0, sizeof q);
    q.a = a;
    q.n = n;
    q.grain = grain;
    q.cap = 64;
    q.first_pivot = first_pivot;
    q.stk = (int64_t *)malloc((size_t)q.cap * 2 * sizeof(int64_t));
    if (!q.stk)
        return -2;
    pthread_mutex_init(&q.mu, NULL);
    pthread_cond_init(&q.cv, NULL);
    (void)SFX(oracle_push)(&q, 0, n - 1);
    pthread_t th[256];
    const int nth = threads > 256 ? 256 : threads;
    int started = 0;
    for (int t = 1; t < nth; t++) {
        if (pthread_create(&th[started], NULL, SFX(oracle_worker), &q) != 0)
            break;
        started++;
    }
    SFX(oracle_worker)(&q);  /* the calling thread works too */
    for (int t = 0; t < started; t++)
        pthread_join(th[t], NULL);
    pthread_cond_destroy(&q.cv);
    pthread_mutex_destroy(&q.mu);
    free(q.stk);
    return q.rc;
}

/* One application of Steps 1-4 to each listed segment. */
int SFX(ksort_oracle_partition_level)(KEY_T *a, const int64_t *left,
                                      const int64_t *len, int64_t nseg,
                                      int64_t *pivot)
{
    for (int64_t s = 0; s < nseg; s++) {
        if (len[s] < 1)
            return -1;
        pivot[s] = SFX(ksort_oracle_partition)(a, left[s], left[s] + len[s] - 1, NULL);
    }
    return 0;
}

/* Steps 1-6 applied to each array of a packed batch on its own. */
int SFX(ksort_oracle_segmented)(KEY_T *a, const int64_t *offsets, int64_t nseg,
                                int64_t *first_pivots)
{
    for (int64_t s = 0; s < nseg; s++) {
        int64_t fp = -1;
        int rc = SFX(ksort_oracle_sort)(a + offsets[s], offsets[s + 1] - offsets[s],
                                        &fp, NULL, 0, NULL, NULL);
        if (rc)
            return rc;
        if (first_pivots)
            first_pivots[s] = fp;
    }
    return 0;
}
